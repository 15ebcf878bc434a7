// Internal plan structures shared by the host code and the HIP kernels.
//
// Notation: sparse level L, finest level J = L-1, N = 2^J fine intervals per
// axis of Omega and of (0,T).  Spatial level a has interior nodes
// K = 1..2^a-1 per axis (array index K-1); fine positions are p = 0..N with
// interior p = 1..N-1 (array index p-1).  Time level b has nq = 2^b+1 nodes
// (P1 nodes t_q = q T/2^b) or spline coefficients (psi_i = B_{i+1}).
//
// A "channel" is one component (a, b) of the combination attached to its
// spatial level a, together with a tap table that says how fine time slab n
// couples to the component's time index q:   sum_k w[n][k] * X[q0[n]+k].
// Two tap families exist:
//   * P1 taps  (Lambda_b^T M_e)[q][n]: the fine weighted P1 mass M_e followed
//     by full-weighting to the P1 nodes of level b (load of eq. (9));
//   * spline taps psi^b_q(t_n): evaluation of level-b splines at fine nodes
//     (prolongation of component solutions, eq. (19)).
// Tables satisfy 0 <= q0[n] <= nq-3 and q0[n+1]-q0[n] in {0,1}.
#pragma once

#include <cstdint>

namespace sg {

constexpr int kMaxLevels = 16;  // J <= 15
constexpr int kChannels = 2;    // channels per spatial level

struct Channel {
  int active;        // 0 or 1
  int a;             // spatial level
  int nq;            // number of time nodes / coefficients
  int qb;            // time capacity of one partial block (restriction)
  const int *q0;     // [ntf]
  const double *w;   // [ntf][3]
  double *data;      // restriction: output Z[nq][nsp]; prolongation: input Y[nq][nsp]
  long long part_off;// offset of this channel's partial blocks (doubles)
  double scale;      // factor applied to this channel's contribution
  int pad;
};

struct Geometry {
  int d;        // 1 or 2
  int J;        // finest level
  int N;        // 2^J
  int nxf;      // N - 1
  int ntf;      // N + 1
  int TS;       // tile side (fine positions)
  int lts;      // log2(TS)
  int ntile;    // tiles per axis = N / TS
  int R;        // deepest in-tile level offset r = J - a  (min(lts, J-1))
  int A0;       // coarsest in-tile spatial level = J - R
  int chunk;    // fine slabs per time chunk
  int nchunk;   // number of chunks
  int phase;    // chunk c covers slabs [c chunk - phase, (c+1) chunk - phase) within
                // [0, ntf): shifts the chunk starts onto the slabs where the finest
                // level's time window moves (a coarsest level above 1)
};

// Slabs [n0, n1) of time chunk c.
__host__ __device__ inline void chunk_span(const Geometry &g, int c, int &n0, int &n1) {
  const int a = c * g.chunk - g.phase;
  n0 = a > 0 ? a : 0;
  n1 = a + g.chunk < g.ntf ? a + g.chunk : g.ntf;
}

// Number of in-tile nodes per axis at level offset r (r = J - a).
//   mode 0: region [TS t, TS t + TS - 1] (restriction and plain prolongation)
//   mode 1: region [TS t - 1, TS t + TS] (prolongation followed by a stencil)
__host__ __device__ inline int tile_nodes(int TS, int r, int mode) {
  if (r == 0) return TS + 2 * mode;
  return (TS >> r) + 1 + mode;
}

// First in-tile node (global position at level offset r) of tile t.
__host__ __device__ inline int tile_lo(int TS, int t, int r, int mode) {
  int p = TS * t - mode;  // may be -1
  // floor division by 2^r for possibly negative p
  return p >= 0 ? (p >> r) : -(((-p) + (1 << r) - 1) >> r);
}

struct KernelTables {
  // per time level b (1..J): banded A_b, B_b [nq][5] (columns i-2..i+2)
  const double *A[kMaxLevels + 1];
  const double *B[kMaxLevels + 1];
  const double *Alo[kMaxLevels + 1];  // low parts of the double-double entries
  const double *Blo[kMaxLevels + 1];
  // derivative values D_b[i][q] for q = i (dlo) and q = i+1 (dhi)
  const double *Dlo[kMaxLevels + 1];
  const double *Dhi[kMaxLevels + 1];
  // g_b[i] = int psi_i' e^{-t/T} dt
  const double *g[kMaxLevels + 1];
  // 1-D P1 eigenvalues at spatial level a: m_k, kappa_k (unit c), k=1..2^a-1
  const double *m1[kMaxLevels + 1];
  const double *k1[kMaxLevels + 1];
};

}  // namespace sg
