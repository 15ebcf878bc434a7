// Kernel argument structures and launch wrappers (host side declarations).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace sg {

// Channel table passed by value (kernel argument segment): the streaming
// kernels read it through scalar loads that cannot alias their stores.
constexpr int kChanMax = 2 * kMaxLevels;

// Per-slab tap of one in-tile channel (2-D passes with 16 x 16 tiles): the
// weights of the three open time nodes and
//   restriction:   the partial-block offset (channel offset + chunk-relative
//                  row) of the node that closes at this slab, -1 if none;
//   prolongation:  the new first time index q0 if the coefficient window
//                  moves on by one at this slab, else -1 (the weights include
//                  the channel sign).
// Entry 0 (the level-J channel, whose window never moves) holds instead the
// bit mask of the entries li whose base is set at this slab.
// One table per pass, [ntf][2 (lts + 1)].
struct TapEntry {
  double w[3];
  long long base;
};

// ---- fine-grid streaming restriction ------------------------------------
// Z_c[q][K] = sum_n sum_m w_c(n,q) phi^a_K(x_m) (S X_n)[m] for every active
// channel c, S = identity or the fine mass matrix (stencil = 1).
struct RestrictArgs {
  Geometry g;
  const double *X;       // [ntf][nxf^d]
  int stencil;           // 0 identity, 1 mass
  double sx, sy;         // h_x/6, h_y/6 of the finest mesh
  double *part;          // partial blocks of the in-tile levels
  double *coarse;        // per-slab partials at level A0 (if A0 > 1)
  const TapEntry *taps;  // per-slab taps of the in-tile channels (16 x 16 tiles only)
  const int *safe_q0;    // tap tables of some active channel: a valid address
  const double *safe_w;  // for loads whose result is discarded
  Channel ch[kChanMax];  // channel (a-1)*2+k, entries >= 2J unused
};

// ---- fine-grid streaming prolongation ------------------------------------
// out[n][m] (+)= base[m] + S( sum_c scale_c sum_q w_c(n,q) (Phi_a Y_c[q])(x_m) )
struct ProlongArgs {
  Geometry g;
  const double *coarse;  // C[n][(2^A0-1)^d] (if A0 > 1)
  const double *base;    // [nxf^d] or null
  double *out;           // [ntf][nxf^d]
  int accumulate;        // 1: add to existing out
  int stencil;           // 0 none, 1 mass
  double sx, sy;
  const int *safe_q0;    // tap tables of some active channel (valid addresses)
  const double *safe_w;
  const TapEntry *taps;  // per-slab taps of the in-tile channels (16 x 16 tiles only)
  Channel ch[kChanMax];
};

struct WorkItem {        // flattened per-channel work (reduce / coarse kernels)
  int ch;                // channel index
  int pad;
  long long start;       // first global element
  long long count;
};

// ---- one stage of many problems in one launch ------------------------------
// Member m of the launch runs blocks [first[m], first[m] + nblk[m]) (first[m]
// a multiple of 8, so the streaming kernels' XCD-aware block order holds per
// member) with its argument struct args[m]; the data pointers that change
// from call to call come from the call's table ptr[slot * nprob + prob[m]]
// for the slots the stage reads (-1: the argument struct's own pointer).
// Pointer slots of a batch call:
enum BatchSlot { kSlotF = 0, kSlotU0, kSlotV0, kSlotU, kSlotG, kSlotDF, kSlotDU0, kSlotDV0,
                 kBatchSlots };
struct ManyLaunch {
  const void *args;          // device array of argument structs
  const int *first;          // [n + 1]
  const int *nblk;           // [n]
  const int *prob;           // [n] member -> problem index
  const double *const *ptr;  // device pointer table [kBatchSlots][nprob]
  int n, nprob;
  int s0, s1, s2, s3;        // slots of the stage's per-call pointers (meaning per kernel)
};

// argument structs of the flat and per-slab kernels in launches of many problems
struct ReduceArgs {      // k_reduce / k_coarse_restrict
  Geometry g;
  const Channel *ch;
  const double *in;      // partial blocks (reduce) or per-slab restrictions SL (coarse)
  const WorkItem *items;
  int nitems;
  long long total;
};
struct CoarseArgs {      // k_coarse_pyramid (in = coarse partials, out = SL) and
  Geometry g;            // k_prolong_coarse (ch, out = the level-A0 array)
  const Channel *ch;
  const double *in;
  double *out;
};
struct StencilArgs {     // k_fine_stencils
  int N, mode;
  const double *ce;
  double hx, hy;
  const double *v, *u;
  double *mv, *ku;
  const double *gsum;
};


// MFMA GEMM tiles: SG_GEMM_W x SG_GEMM_W waves per workgroup, each a 32 x 32
// sub-tile (tiles of 32 SG_GEMM_W square)
#ifndef SG_GEMM_W
#define SG_GEMM_W 2
#endif
constexpr int kGemmTile = 32 * SG_GEMM_W;
constexpr int kGemmThreads = 64 * SG_GEMM_W * SG_GEMM_W;

struct GemmDesc {
  const double *A;
  const double *B;
  double *C;
  int M, N, K;
  int lda, ldb, ldc;
  long long sA, sB, sC;
  int batch, tm, tn;
  int tile0;
  // folded transforms (launches with fold 1 or 2; a DST-I matrix Q of odd
  // order nref, whose entry (k, j) and entry (nref-1-k, j) differ by the sign
  // (-1)^j): the sum over k in C = A B runs over the pairs k, nref-1-k of A's
  // columns (fold 1) or B's rows (fold 2), added for the outputs j of even
  // parity (par 0, k = 0..nref/2 with the middle index unpaired) and
  // subtracted for odd ones (par 1, k < nref/2); C's columns (fold 1) or rows
  // (fold 2) are the outputs 2 j' + par
  int nref, par;
  // transposed operands (plain products only): ta, element (i, k) of A at
  // k lda + i; tb, element (k, j) of B at j ldb + k.  A list is launched
  // with the k_gemm variant of its operands (FOLD 3 for ta, 4 for tb), and
  // its descriptors all share the flag (checked when the list is uploaded)
  int ta, tb;
};

struct ModeTables {      // 1-D P1 eigenvalues per level and axis (unit c)
  const double *mx[kMaxLevels + 1];
  const double *kx[kMaxLevels + 1];
  const double *my[kMaxLevels + 1];
  const double *ky[kMaxLevels + 1];
};

struct SolveDesc {
  double *rhs;           // [nq][nmodes], overwritten with the solution
  double *fac;           // 5 planes [nq][nmodes]: L1, L2, 1/U0, U1, U2 of E = L U
  double *scratch;       // 2 planes [nq][nmodes]
  int nq, nmodes;
  int b, a;              // time level, spatial level
  int refine;            // maximum refinement sweeps (double-double residual)
  int transpose;         // solve with the transposed time matrices
  int wave;              // 1: one wave per mode (long time levels), 0: one thread
  int flat;              // 1: modes of a dense spatial pencil (2-D variable speed):
                         //    mass mx[a][j], stiffness c2 kx[a][j], as in 1-D
  double c2;             // wave speed squared (constant-speed path)
  long long thread0;     // first global thread, a multiple of 64 (one wave
                         // never spans two descriptors)
  const KernelTables *kt;  // the problem's time tables
  const ModeTables *mt;    // and spatial mode tables
  int d;                   // its dimension
  int pad2;
};

// One component of a 1-D variable-speed problem solved without a spatial
// eigenbasis: block LU of S = A (x) M + B (x) K in space-major order (blocks
// of nq x nq, one per spatial node) as an approximate inverse, refined with
// the double-double residual of the whole component system.
struct BlockDesc {
  const double *in;      // right-hand side [nq][nx]
  double *out;           // solution [nq][nx]
  const double *Dinv;    // [nx][nq][nq] inverses of the block pivots D_k
  const double *Lf;      // [nx][nq][nq] multipliers L_k = S_{k,k-1} D_{k-1}^{-1} (k >= 1)
  const double *mk;      // [nx][kSpaceStride]: M_kk, M_{k,k+1}, K_kk, K_{k,k+1}, low parts of
                         // K_kk, K_{k,k+1} (coupling entries zero at k = nx-1)
  double *work;          // 3 planes [nq][nx]: saved rhs, residual, intermediate vector
  int nq, nx, b;         // time nodes, spatial nodes, time level
  int transpose;         // solve with S^T
  int refine;            // maximum refinement sweeps
  int pad;
  const KernelTables *kt;  // the problem's time tables
};


struct CompDesc {        // one component for the small post-processing kernels
  double *data;          // output [nq][nsp]: load b_c, or adjoint zeta_c
  const double *z;       // input [nq][nsp]: restricted data Z_c, or adjoint z_c
  const double *mv;      // level-a field Phi^T M v0 (load only)
  const double *ku;      // level-a field Phi^T K u0 (load only)
  int a, b, nq, nsp;
  int sign;
  int pad;
  long long start;       // first global element of this component's work
  const KernelTables *kt;  // the problem's time tables
};

struct LevelDesc {       // adjoint fields of one spatial level
  int a, nsp;
  int c0, c1;            // component indices at this level (-1 if none)
  double *fv;            // sum_c psi_0'(0) z_c[0]
  double *fu;            // sum_c sum_i g_c[i] z_c[i]
  int wave;              // 1: one wave per node (long time sums), 0: one thread
  int pad;
  long long start;       // first global thread (a multiple of 64 for wave levels)
  const CompDesc *cd;    // the problem's adjoint component list (c0, c1 index it)
  const KernelTables *kt;  // the problem's time tables
};

// launch wrappers (return hipError_t of the launch)
hipError_t launch_restrict(const RestrictArgs &a, hipStream_t s);
hipError_t launch_reduce(const Geometry &g, const Channel *ch, const double *part,
                         const WorkItem *items, int nitems, long long total,
                         hipStream_t s);
// launches of many problems (ManyLaunch.args holds RestrictArgs /
// ProlongArgs / ReduceArgs / CoarseArgs / StencilArgs); proto: any member's
// arguments (the kernel variant: dimension, tile, stencil, finest channels);
// slots: restrict X = s0; prolong base = s0, out = s1; stencils v = s0,
// u = s1, mv = s2, ku = s3 (-1: the struct's own)
hipError_t launch_restrict_many(const RestrictArgs &proto, const ManyLaunch &M, int blocks,
                                hipStream_t s);
hipError_t launch_prolong_many(const ProlongArgs &proto, const ManyLaunch &M, int blocks,
                               hipStream_t s);
hipError_t launch_reduce_many(const Geometry &proto, const ManyLaunch &M, int blocks,
                              hipStream_t s);
hipError_t launch_coarse_pyramid_many(int d, const ManyLaunch &M, int blocks, hipStream_t s);
hipError_t launch_coarse_restrict_many(int d, const ManyLaunch &M, int blocks, hipStream_t s);
hipError_t launch_prolong_coarse_many(int d, const ManyLaunch &M, int blocks, hipStream_t s);
hipError_t launch_fine_stencils_many(int d, const ManyLaunch &M, int blocks, hipStream_t s);
// largest level-A0 array (nodes) the coarse pyramid kernel holds in LDS
constexpr int kCoarseMax = 4096;
// per-slab level-A0 values assembled from the restriction's per-slab tile
// partials (coarse_part), restricted to the levels a < A0:
// SL[n][off_a + K], off_a = sum_{a' < a} (2^a' - 1)^d
hipError_t launch_coarse_pyramid(const Geometry &g, const double *coarse_part, double *SL,
                                 hipStream_t s);
hipError_t launch_coarse_restrict(const Geometry &g, const Channel *ch,
                                  const double *SL, const WorkItem *items,
                                  int nitems, long long total, hipStream_t s);
hipError_t launch_prolong_coarse(const Geometry &g, const Channel *ch,
                                 double *C, int mode, hipStream_t s);
hipError_t launch_prolong(const ProlongArgs &a, hipStream_t s);
// Energy 1/2 ||ut_k||^2 + 1/2 ||c grad w_k||^2 of K finest-mesh slabs into E[k]
// (part: K * nblk doubles of block partial sums).
hipError_t launch_energy(int d, int N, const double *ce, double hx, double hy, const double *W,
                         const double *Ut, int K, int nblk, double *part, double *E,
                         hipStream_t s);
// fused energy of u_h (2-D, 16 x 16 tiles): value pass a (base = u0), the
// derivative pass's taps and coarse array; part[K][ntile^2], then E[K]
hipError_t launch_energy_w(const ProlongArgs &a, const TapEntry *taps_d, const double *coarse_d,
                           const double *ce, double hx, double hy, double *part, int K,
                           int ntile2, double *E, hipStream_t s);
// L^2(Q_T) error by quadrature: W [K][n^d] u_h at the Gauss instants, uq
// [K][(2N)^d] the exact solution at the Gauss points; out[0] = int (u - u_h)^2,
// out[1] = int u^2 (wt: the time weights of the instants); part [K][nblk][2]
hipError_t launch_l2(int d, int N, double hx, double hy, const double *W, const double *uq,
                     int K, int nblk, double *part, const double *wt, double *out,
                     hipStream_t s);
hipError_t launch_fine_stencils(int d, int N, const double *ce, double hx,
                                double hy, const double *v_in, const double *u_in,
                                double *mv_out, double *ku_out,
                                const double *gsum, int mode, hipStream_t s);
hipError_t launch_post_load(const CompDesc *cd, int ncomp, long long total, hipStream_t s);
hipError_t launch_post_adjoint(const CompDesc *cd, int ncomp, long long total, hipStream_t s);
hipError_t launch_adjoint_fields(const LevelDesc *ld, int nlev, long long total, hipStream_t s);
hipError_t launch_gemm(const GemmDesc *descs, int ndesc, int total_tiles, int fold,
                       hipStream_t s);
hipError_t launch_time_factor(const SolveDesc *sd, int nsd, long long total, hipStream_t s);
// transpose: every descriptor of the list solves the transposed (adjoint)
// systems (SolveDesc.transpose), else none does
hipError_t launch_time_solve(const SolveDesc *sd, int nsd, long long total, int transpose,
                             hipStream_t s);
hipError_t launch_block_solve(const BlockDesc *bd, int nbd, hipStream_t s);
// ---- 2-D variable-speed components of short time levels -------------------
// S = A (x) M + B (x) K(c) is diagonalised in time (B^{-1} A = V diag(lam)
// V^{-1}), leaving one complex spatial system (lam M + K(c)) w = r per
// eigenvalue (one of each conjugate pair).  Each is solved directly by
// splitting Omega into the ns strips of wave-speed blocks along y: inside a
// strip c depends on x only, so a sine transform along the strip's m interior
// rows diagonalises the y direction and leaves one tridiagonal system in x
// per y mode,
//   T_{k,l} = mu_l (lam M_x + K_x^k) + nu_l M_x^k,
// (K_x^k, M_x^k the c^2-weighted 1-D stiffness and mass of strip k); the
// ni = ns - 1 interface rows between strips carry a dense Schur complement,
// inverted at assembly.  Complex values are interleaved (re, im).
struct FdmDesc {
  const double *in;      // right-hand side [nq][n][n] (real)
  double *out;           // solution [nq][n][n] (real)
  const double *tin;     // time transform in, complex [nu][nq]
  const double *tout;    // time transform out, complex [nq][nu]
  const double *lam;     // eigenvalues, complex [nu]
  double *X, *Y;         // complex [nu][n][n] work arrays: X row-major (y, x); Y holds each
                         // strip's y-transformed values mode-fastest, [x][re, im][l] from the
                         // strip's first row (X's strip rows likewise during the correction)
  double *E;             // complex [nu][ns][2][n]: strip solutions at their first / last row
  double *G;             // complex [nu][ni][n]: interface right-hand sides
  double *Xg;            // complex [nu][ni][n]: interface solutions
  double *Sinv;          // complex [nu][ni n][ni n]: inverse interface Schur complements
  double *fac;           // 3 complex planes [nu][ns][n][m]: 1/d'_x, the multiplier l_x (top-down LU of T_{k,l}), 1/d''_x (bottom-up)
  const double *xt;      // [ns][4][n]: K_x^k diagonal, coupling (x, x+1); M_x^k diagonal, coupling
  const double *ym;      // [3][m]: mu_l, nu_l, s_l(first row) of the strip sine transform
  int nq, n, nu, ns, m, ni;
  double hx, hy;
  long long node0;       // first thread: time transforms (n^2 per descriptor)
  long long tri0;        // first thread: tridiagonal solves (nu ns m)
  long long edge0;       // first thread: strip edge rows (nu ns n)
  long long if0;         // first thread: interface right-hand sides (nu ni n)
  long long gemv0;       // first wave: interface solves (nu ni n rows)
};

// most eigenvalues kept per time level (2^4 + 1 = 17 nodes: 8 pairs + 1 real)
constexpr int kFdmMaxNu = 9;

struct FdmTotals {       // launch sizes of one list of FdmDesc
  long long node = 0, tri = 0, edge = 0, iface = 0, gemv = 0;
};

// solve phase of a list of components (stream ordered; the strip sine
// transforms are the GEMM lists gf (X -> Y) and gi (Y -> X))
hipError_t launch_fdm_in(const FdmDesc *d, int nd, const FdmTotals &t, hipStream_t s);
// chunk: rows per register chunk of the sweeps (4, 8 or 16)
hipError_t launch_fdm_tri(const FdmDesc *d, int nd, const FdmTotals &t, int correction,
                          int chunk, hipStream_t s);
hipError_t launch_fdm_interface(const FdmDesc *d, int nd, const FdmTotals &t, hipStream_t s);
hipError_t launch_fdm_out(const FdmDesc *d, int nd, const FdmTotals &t, hipStream_t s);
// assembly of one component (descriptor h, device pointers): tridiagonal
// factors, strip Green's functions at the rows next to the interfaces, the
// interface Schur complements and their inverses (Gauss-Jordan, partial
// pivoting).  Allocates and frees its temporaries; synchronises the device.
hipError_t fdm_assemble(const FdmDesc &h);

hipError_t launch_fill(double *p, long long n, double v, hipStream_t s);

// Statically allocated scratch for callers that cannot allocate device
// memory: one array per device, kStaticScratchDoubles doubles (64 MiB), held
// until the process ends.  static_scratch returns the current device's copy
// (its address is looked up once per device, with that device current).
// Every call that uses it on one device shares it: such calls must not
// overlap.
constexpr long long kStaticScratchDoubles = (64LL << 20) / 8;
hipError_t static_scratch(double **ptr);
hipError_t launch_broadcast(double *out, const double *base, int nt, long long nsp,
                            hipStream_t s);

}  // namespace sg
