/*
 * sgwave.h - C ABI of the MI355X space-time sparse-grid wave solver.
 *
 * The library computes the sparse-grid combination solution of the linear
 * wave equation (Ferrari, Moiola, Perinati, Perugia, "A space-time
 * sparse-grid method for the wave equation"):
 *
 *   problem (1):     u_tt - div(c^2 grad u) = f on Omega x (0,T), u = 0 on the
 *                    boundary, u(0) = u0, u_t(0) = v0;
 *   component solve: the Galerkin problem (9) on V^x_{jx} (x) V^t_{jt}
 *                    (P1 / Q1 in space, quadratic C^1 splines with w(0) = 0 in
 *                    time, exponentially weighted coercive form (6));
 *   combination:     eq. (19), +1 on jx+jt = L and -1 on jx+jt = L-1
 *                    (jx, jt >= 1), plus the lift by u0 (Sec. 2.1).
 *
 * Level convention: level j has 2^j uniform intervals per axis of Omega and
 * of (0,T); the finest level of sparse level L is J = L-1 (the paper's J is
 * L-2 with h_0 = 1/2).
 *
 * Data layout (all buffers FP64, contiguous, device memory, caller-owned):
 *   fine space-time array  [nt][ny][nx]  x fastest; nt = 2^J + 1 time nodes
 *                          t_n = n T / 2^J including t = 0 and t = T;
 *                          nx = ny = 2^J - 1 interior nodes (ny = 1 when d = 1);
 *                          values on the spatial boundary are implicitly 0.
 *   fine space array       [ny][nx].
 * Input data are read as nodal values of their piecewise-linear (P1 in time,
 * P1/Q1 in space) interpolants on the finest grid.  The output U holds the
 * nodal values of u^CF + u0; U[0] equals u0.
 *
 * Ownership: the caller owns every data buffer; the library owns the handle,
 * its tables and its device workspace (allocated once in sg_assemble).
 * sg_solve / sg_adjoint never allocate, never synchronise the host, and are
 * stream ordered; one handle must not be used by two streams at once.
 * Errors are returned as status codes; sg_last_error() gives a message for
 * the calling thread.  No C++ exception crosses this interface.
 */
#ifndef SGWAVE_H
#define SGWAVE_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_problem sg_problem;

typedef enum {
  SG_OK = 0,
  SG_EINVAL = -1,   /* invalid argument (sizes, c <= 0, T <= 0, L < 2, NULL) */
  SG_ENOMEM = -2,   /* device or host allocation failed (assemble only)      */
  SG_EDEVICE = -3,  /* a HIP runtime call failed                             */
  SG_ENOTSUP = -4,  /* configuration outside what the library implements   */
  SG_ESTATE = -5    /* call not valid in the handle's current state          */
} sg_status;

/*
 * Build the discrete operator of problem (1) for sparse level L.
 *   d       spatial dimension, 1 or 2.
 *   len     side lengths of Omega = (0,len[0]) [x (0,len[1])], host pointer.
 *   ncell   number of uniform wave-speed blocks per axis, host pointer.
 *   c_vals  c on the blocks (x fastest), ncell[0]*ncell[1] values > 0, host.
 *           2^(L-1) must be a multiple of every ncell[i] (the finest mesh
 *           resolves the blocks).
 *   T       final time > 0.   L  sparse level, 2 <= L <= 16.
 * On success *out receives a handle bound to the current HIP device; all
 * tables are uploaded and all workspace is allocated here.  A wave speed
 * that varies in 2-D is handled per component: spatial levels <= 5 (and 6
 * with more than 17 time nodes) through the dense pencil (K(c), M),
 * diagonalised here with rocSOLVER; spatial levels >= 6 with at most 17 time
 * nodes by diagonalising the time matrices and solving each shifted spatial
 * system directly by strips of wave-speed blocks (at least two mesh rows per
 * block along y, at most 4096 interface nodes).  A component outside both
 * (e.g. spatial level 7 with 33 time nodes, L >= 12), and 1-D variable speed
 * on spatial levels >= 9 with more than 64 time nodes: SG_ENOTSUP.
 */
sg_status sg_assemble(int d, const double *len, const int *ncell,
                      const double *c_vals, double T, int L, sg_problem **out);

/*
 * sg_assemble with the coarsest level of the combination as a parameter: the
 * coarse-mesh study of Sec. 6.3 (Fig. 10) varies the level-0 mesh size h_0.
 * Level j of this library has 2^j uniform intervals, so h_0 = 2^-b0 of the
 * domain side and of T; the components are eq. (19) with its levels shifted
 * by b0 and the finest level kept at L-1:
 *   {(jx, jt) : jx, jt >= b0, jx + jt in {L-1+b0, L-2+b0}},
 * 2(L-1-b0)+1 of them, +1 on the first diagonal and -1 on the second.
 *   b0      1 <= b0 <= L-1 (b0 = 1 is sg_assemble; b0 = L-1 is the single
 *           full-grid component (L-1, L-1)); otherwise SG_EINVAL.
 * Every other argument, the limits and the returned handle are those of
 * sg_assemble.  The streaming passes cut their time chunks where the finest
 * spatial level's time window moves (its component has time level b0), so
 * a large b0 makes the chunks short.
 */
sg_status sg_assemble_offset(int d, const double *len, const int *ncell,
                             const double *c_vals, double T, int L, int b0,
                             sg_problem **out);

/*
 * Forward solve: U = u0 + sum_c s_c P_c(f, u0, v0) on the finest grid
 * (component solves of eq. (9), combination eq. (19), lift).  f and U are
 * fine space-time arrays, u0 and v0 fine space arrays (device pointers).
 * This is the fused path: one streaming pass over f, batched component
 * solves, one streaming pass writing U.  U may not alias f.
 */
sg_status sg_solve(sg_problem *p, const double *f, const double *u0,
                   const double *v0, double *U, hipStream_t stream);

/*
 * The same result computed by the literal per-component loop: for each
 * component, restrict from f, solve, and accumulate into U (2 fine-grid
 * passes per component).  Reference point for the fused path's speedup.
 */
sg_status sg_solve_plain(sg_problem *p, const double *f, const double *u0,
                         const double *v0, double *U, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): sg_solve with
 * its per-call scratch (partial sums of the streaming restriction, the
 * coarse-level arrays and two fine space fields) taken from a statically
 * allocated device array of 64 MiB instead of the handle's workspace.  Same
 * arguments, arithmetic and result as sg_solve, bit for bit.  Allocates
 * nothing and calls no allocating routine.  The array exists once per device
 * and is shared by every call on that device: calls that overlap on one
 * device (any handles, any streams) race and must be ordered by the caller.
 * It keeps the last call's contents; the call clears what must start at zero
 * itself.  SG_ENOTSUP (message states the need) if the problem needs more
 * than 64 MiB of scratch; SG_ESTATE if the current device is not the
 * handle's.
 */
sg_status sg_solve_static(sg_problem *p, const double *f, const double *u0,
                          const double *v0, double *U, hipStream_t stream);

/*
 * Adjoint of the forward map F: (f,u0,v0) -> U.  g has the layout of U;
 * df the layout of f; du0, dv0 fine space arrays.  Computes
 * (df, du0, dv0) = F^T g (transposed combination, transposed component
 * solves, transposed load).  Any output pointer may be NULL to skip it.
 */
sg_status sg_adjoint(sg_problem *p, const double *g, double *df, double *du0,
                     double *dv0, hipStream_t stream);

/*
 * Capture sg_solve (and, if g != NULL, sg_adjoint) for fixed buffers into a
 * HIP graph owned by the handle, replacing any earlier capture.  The stream
 * must not be capturing already.  sg_graph_launch replays it on a stream.
 * With a given cotangent the adjoint does not depend on the forward; it
 * keeps its own workspace and runs on a parallel branch of the graph, unless
 * an output of one direction is a buffer of the other, or stage events are
 * set (sg_set_events: their kernels are timed alone); then one after the
 * other.
 */
sg_status sg_graph_capture(sg_problem *p, const double *f, const double *u0,
                           const double *v0, double *U, const double *g,
                           double *df, double *du0, double *dv0,
                           hipStream_t stream);
sg_status sg_graph_launch(sg_problem *p, hipStream_t stream);

/*
 * Stage timing: when ev is not NULL, sg_solve and sg_adjoint record
 * ev[i] (caller-created hipEvent_t, at least SG_NUM_EVENTS of them) on the
 * call's stream at these points; a NULL entry leaves its point out.  When
 * sg_graph_capture runs, the pairs (1, 2), (5, 6), (8, 9) and (12, 13) whose
 * two events are both set become event-record nodes around their kernel,
 * recorded by every replay (each node costs a few microseconds of the
 * replay, so a caller timing replays sets only the pairs it reads):
 *   0 forward begin        1 before the load restriction   2 after it
 *   3 before the solves    4 after the solves              5 before the
 *   combination pass       6 after it (forward end)
 *   7 adjoint begin        8 before the cotangent restriction 9 after it
 *  10 before the solves   11 after them   12 before the df pass 13 after it
 *  14 adjoint end
 * Pass ev = NULL to stop recording.
 */
#define SG_NUM_EVENTS 15
sg_status sg_set_events(sg_problem *p, hipEvent_t *ev, int n);

/*
 * Sizes: nt = 2^J+1, n = 2^J-1 interior nodes per axis, n_sparse = sum of
 * the component dimensions (the paper's N^sparse_DoFs), n_full = nt * n^d.
 * Any output pointer may be NULL.
 */
sg_status sg_query(const sg_problem *p, int *nt, int *n, long long *n_sparse,
                   long long *n_full, int *n_components);

/*
 * Component c (0 <= c < n_components): levels, sign and dimensions.  The
 * order is the library's internal order (stable for a given L).
 */
sg_status sg_component_info(const sg_problem *p, int c, int *jx, int *jt,
                            int *sign, int *n_space, int *n_time);

/*
 * Copy the coefficients of component c into host memory `out` of
 * n_time * n_space doubles (time index outer); synchronises the device.
 * stage 0: right-hand side b_c of eq. (9) of the last sg_solve;
 * stage 1: its solution u_c;  stage 2: the adjoint right-hand side
 * s_c Psi^T g Phi of the last sg_adjoint;  stage 3: its solution
 * S_c^{-T} (s_c Psi^T g Phi).  For tests of intermediate stages.
 */
sg_status sg_component_copy(sg_problem *p, int c, int stage, double *out);

/*
 * Host-only introspection of the tables the library builds (no device use).
 * sg_host_time_level: time matrices of level b on (0,T) (Prop. 1, eq. (30)):
 *   A, B   banded [2^b+1][5], entry (i, j) at [i][j-i+2] (high parts);
 *   Alo, Blo low parts: A + Alo, B + Blo hold the entries to about 32 digits;
 *   Dlo,Dhi psi_i'(t_i), psi_i'(t_{i+1}) at the level-b nodes;
 *   g      int_0^T psi_i' e^{-t/T} dt.   Each array holds 2^b+1 rows.
 * sg_host_taps: tap table of level b on the fine time grid of level J
 *   (kind 0: P1 load taps, kind 1: spline evaluation taps): q0[2^J+1],
 *   w[3*(2^J+1)]; slab n couples to time index q0[n]+k with weight w[3n+k].
 * Any output pointer may be NULL.
 */
sg_status sg_host_time_level(int b, double T, double *A, double *Alo, double *B,
                             double *Blo, double *Dlo, double *Dhi, double *g);
sg_status sg_host_taps(int kind, int b, int J, double T, int *q0, double *w);

/*
 * The time chunks a streaming pass uses when the finest level's channel has
 * the window q0 (ntf host values, one per slab; e.g. from sg_host_taps):
 * starting from chunks of `chunk` slabs, the longest chunk length whose
 * starts, shifted back by a phase, fall on every slab where q0 moves (the
 * kernels keep the finest level's coefficients fixed within a chunk).  Chunk
 * c covers slabs [c*chunk - phase, (c+1)*chunk - phase) within [0, ntf).
 * Outputs (host): *out_chunk, *out_phase, *out_nchunk.  Host only.
 */
sg_status sg_host_time_chunks(int ntf, int chunk, const int *q0, int *out_chunk,
                              int *out_phase, int *out_nchunk);

/*
 * Energy of the computed solution (Sec. 6.3, the energy diagnostic):
 *   E(t) = 1/2 ||d_t u_h(t)||^2_{L2(Omega)} + 1/2 ||c grad u_h(t)||^2_{L2(Omega)}
 * for u_h = u^CF + u0, the lifted combination solution of the last sg_solve
 * (or sg_solve_plain) on this handle: its component solutions stay in the
 * handle's workspace until the next forward solve (sg_adjoint does not touch
 * them).  u_h(t) is a P1 / Q1 function on the finest mesh, so the integrals
 * are exact (element mass and stiffness forms with the per-block c^2).
 *
 * sg_energy_setup: K >= 1 instants t (host array) in [0, T], ascending, no
 *   two consecutive instants more than one finest time interval T / 2^J
 *   apart (a uniform grid of at least 2^J + 1 instants qualifies; SG_EINVAL
 *   otherwise).  Builds the evaluation tables (spline values and derivatives
 *   of every time level at the instants) and allocates the workspace:
 *   in 2-D with 16 x 16 streaming tiles (J <= 10) the element forms are
 *   applied inside the evaluation: the workspace is one partial sum per
 *   instant and tile and, per instant, the values of the level below the
 *   tiles (each about K (n/16)^2 doubles), and no field is written;
 *   otherwise (1-D, finer 2-D levels) two K x n^d arrays of the fields.  Synchronises the device;
 *   replaces and frees an earlier setup.  SG_ENOMEM if the workspace does not
 *   fit.
 * sg_energy: u0 as given to the forward solve (device, fine space array),
 *   E device array of K doubles (caller-owned).  Stream ordered; allocates
 *   nothing.  SG_ESTATE without a setup.
 */
sg_status sg_energy_setup(sg_problem *p, int K, const double *t);
sg_status sg_energy(sg_problem *p, const double *u0, double *E, hipStream_t stream);

/*
 * L^2(Q_T) error of the computed solution by quadrature (Sec. 6.3, the
 * relative errors of the coarse-mesh study): for an exact solution u given
 * by the caller at the quadrature points,
 *   out[0] = int_{Q_T} (u - u_h)^2,   out[1] = int_{Q_T} u^2,
 * u_h = u^CF + u0 of the last forward solve on this handle (u0 read, like
 * the solver reads it, as its finest-grid interpolant).  The rule is the
 * tensor Gauss rule with 3 points per finest time interval and 2 points per
 * finest element along each space axis: exact for u_h^2 (quadratic in t, Q1
 * in space on every finest cell), of order h^4 for the error integrand.
 * sg_l2_points: the rule (host arrays, any may be NULL): K = 3 * 2^J
 *   instants t[K] with weights wt[K] (ascending), nq = 2 * 2^J points per
 *   space axis xq[nq], yq[nq] (d = 2; the weights are h/2 per point).
 * sg_l2_setup: evaluation tables at the instants and the workspace (one
 *   K x n^d array of u_h at the instants, about 24 * 2^J * n^d bytes);
 *   synchronises the device; replaces an earlier setup.  SG_ENOMEM if it
 *   does not fit.
 * sg_l2_error: u0 as given to the forward solve (device, fine space
 *   array); uq device array [K][nq^d] (d = 2: [K][y][x], x fastest) of u at
 *   the points; out device array of 2 doubles.  Stream ordered; allocates
 *   nothing; a fixed summation order.  SG_ESTATE without a setup.
 */
sg_status sg_l2_points(const sg_problem *p, int *K, double *t, double *wt, int *nq, double *xq,
                       double *yq);
sg_status sg_l2_setup(sg_problem *p);
sg_status sg_l2_error(sg_problem *p, const double *u0, const double *uq, double *out,
                      hipStream_t stream);

/* Release the handle and all device memory it owns.  NULL is accepted. */
sg_status sg_destroy(sg_problem *p);

/* Message describing the last error of the calling thread ("" if none). */
const char *sg_last_error(void);

/*
 * Batches of independent problems (any mix of d, L and wave speeds; the
 * components of every problem are independent, Rem. 2).  A batch references
 * n assembled handles (the caller keeps them alive and owns them).  Every
 * stage runs as ONE launch over all problems per kernel variant, on the
 * caller's stream: each streaming stage (fine stencils, restriction of the
 * data, reductions, coarse levels, prolongation into the outputs) over the
 * block ranges of all problems, longest blocks first; each solve stage
 * (time-diagonalised strip solves, block solves, sine / eigenvector
 * transforms, per-mode time solves, load and adjoint post-passes) over the
 * concatenated work lists of all problems, longest contractions and time
 * levels first.  The per-call data pointers go to the device in a table
 * uploaded by each eager call (stream ordered; the captured graph keeps its
 * own).
 * Argument arrays hold n device pointers each (host arrays).
 * sg_batch_create: builds the merged work lists (allocates device memory).
 * sg_batch_solve / sg_batch_adjoint: the batched forward / adjoint, stream
 *   ordered, allocation-free; results equal each problem's sg_solve /
 *   sg_adjoint bit for bit.  In the adjoint, df, du0, dv0 may be NULL as a
 *   whole or per problem.
 * sg_batch_capture: captures sg_batch_solve (and after it sg_batch_adjoint
 *   when g is not NULL) into one HIP graph owned by the batch;
 *   sg_batch_launch replays it.
 * A handle must not belong to two batches that run at once, nor be used
 * elsewhere while its batch runs.
 */
typedef struct sg_batch sg_batch;
sg_status sg_batch_create(int n, sg_problem *const *problems, sg_batch **out);
sg_status sg_batch_solve(sg_batch *b, const double *const *f, const double *const *u0,
                         const double *const *v0, double *const *U, hipStream_t stream);
sg_status sg_batch_adjoint(sg_batch *b, const double *const *g, double *const *df,
                           double *const *du0, double *const *dv0, hipStream_t stream);
sg_status sg_batch_capture(sg_batch *b, const double *const *f, const double *const *u0,
                           const double *const *v0, double *const *U, const double *const *g,
                           double *const *df, double *const *du0, double *const *dv0,
                           hipStream_t stream);
sg_status sg_batch_launch(sg_batch *b, hipStream_t stream);
/*
 * Measurement support.  sg_batch_info: number of problems, the sum of their
 * component dimensions (N^sparse) and the bytes of the tables one
 * direction's merged solve stages read (inverse interface Schur complements
 * and tridiagonal factors of the strip solves, transform matrices, time-solve
 * LU factors, block-LU factors); outputs may be NULL.
 * sg_batch_set_events: when ev is not NULL (SG_BATCH_EVENTS caller-created
 * events), sg_batch_solve / sg_batch_adjoint record them on the caller's
 * stream at: 0 forward begin, 1 before the merged solves, 2 after them,
 * 3 forward end, 4 adjoint begin, 5 before the merged solves, 6 after them,
 * 7 adjoint end.  Not recorded inside a captured batch graph.
 */
#define SG_BATCH_EVENTS 8
sg_status sg_batch_info(const sg_batch *b, int *n, long long *n_sparse,
                        long long *solve_table_bytes);
sg_status sg_batch_set_events(sg_batch *b, hipEvent_t *ev, int n);
sg_status sg_batch_destroy(sg_batch *b);

/*
 * Host table (exported for tests; no device work): generalised eigenpairs of
 * the level-a P1 pencil (K(c), M) on (0,len) with c piecewise constant on
 * ncell uniform blocks (eq. (9), spatial matrices; variable wave speed in
 * 1-D).  V: (2^a-1)^2 doubles, row-major, column k = eigenvector k with
 * V^T M V = I; lam: 2^a-1 eigenvalues.  Caller-owned host buffers.
 * SG_EINVAL unless 1 <= a <= 8.
 */
sg_status sg_host_pencil(int a, double len, int ncell, const double *c_vals, double *V,
                         double *lam);

/*
 * Host table (exported for tests; no device work): diagonalisation of the
 * time matrices of level b on (0,T) (Prop. 1), B^{-1} A = V diag(lam) V^{-1},
 * used to solve the 2-D variable-speed components of short time levels.
 * Only the real eigenvalues and one member (Im > 0) of each conjugate pair
 * are returned, *nu of them.  Complex arrays are interleaved (re, im);
 * caller-owned host buffers of at least: lam 2*nq, fin/ain 2*nq*nq,
 * fout/aout 2*nq*nq doubles (nq = 2^b + 1).  With P = (B V)^{-1}:
 *   fin[u][j] = P[u][j], fout[j][u] = w_u V[j][u]      (forward solve),
 *   ain[u][j] = V[j][u], aout[j][u] = w_u P[u][j]      (adjoint solve),
 * w_u = 2 for a conjugate pair and 1 for a real eigenvalue, so that
 * S^{-1} b = Re sum_u fout[.][u] (lam_u M + K)^{-1} sum_j fin[u][j] b_j.
 * Any output may be NULL.  SG_EINVAL unless 1 <= b <= 5 and T > 0.
 */
sg_status sg_host_time_fdm(int b, double T, int *nu, double *lam, double *fin, double *fout,
                           double *ain, double *aout);

/*
 * Host table (exported for tests; no device work): the dense level-a Q1
 * pencil in 2-D, K(c) and M of eq. (9) on (0,len[0]) x (0,len[1]) with c
 * piecewise constant on ncell[0] x ncell[1] uniform blocks (x fastest).
 * K, M: caller-owned host buffers of n^4 doubles, n = 2^a - 1, row-major
 * over the interior nodes (x fastest); either may be NULL.  SG_EINVAL unless
 * 1 <= a <= 6.
 */
sg_status sg_host_pencil_2d(int a, const double *len, const int *ncell, const double *c_vals,
                            double *K, double *M);

#ifdef __cplusplus
}
#endif

#endif /* SGWAVE_H */
