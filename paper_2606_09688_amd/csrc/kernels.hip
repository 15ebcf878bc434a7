// HIP kernels for gfx950 (CDNA4), FP64 throughout.
//
// Fine-grid passes (memory bound, one HBM sweep each):
//   k_restrict   streams the fine space-time data slab by slab; per spatial
//                tile it builds the P1 restriction pyramid (full weighting,
//                levels J .. A0) in LDS and accumulates each level into the
//                time nodes of its components with the channel tap tables.
//                Partial sums of nodes shared with neighbouring tiles/chunks
//                go to a scratch buffer; k_reduce adds them in a fixed order
//                (deterministic, no atomics).
//   k_prolong    the transpose structure: per tile and slab it evaluates every
//                component at its own nodes in time (tap tables), interpolates
//                level by level to the fine grid in LDS and writes the
//                combination (+ u0) once.
// Levels coarser than the tile (a < A0) are handled by small gather kernels
// on a per-slab level-A0 array.
//
// Component solves (cache resident): batched DST-I along each space axis as
// FP64 GEMMs with the orthonormal sine matrix, then one banded (pentadiagonal)
// LU per spatial mode of (m_k A_b + kappa_k B_b), optionally refined with a
// double-double residual, then the inverse transforms.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sg {

// ---------------------------------------------------------------- helpers --

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }
__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int D, int TS, int MODE>
struct Shape {
  static constexpr int LTS = ilog2c(TS);
  __host__ __device__ static constexpr int nodes(int r) {
    return r == 0 ? TS + 2 * MODE : (TS >> r) + 1 + MODE;
  }
  __host__ __device__ static constexpr int size(int r) { return ipow(nodes(r), D); }
  __host__ __device__ static constexpr int offset(int r) {
    return r == 0 ? 0 : offset(r - 1) + size(r - 1);
  }
  static constexpr int total = offset(LTS + 1);
  static constexpr int upper = total - ipow(TS + 2 * MODE, D);  // levels r >= 1
  static constexpr int max_upper_size = size(1);
};

__device__ __forceinline__ bool interior(int p, int n) { return p >= 1 && p <= n; }

__device__ __forceinline__ long long gid64() {
  return (long long)blockIdx.x * blockDim.x + threadIdx.x;
}

// --------------------------------------------------------- restriction -----

template <int D, int TS, int TB, int NT>
__global__ void __launch_bounds__(NT) k_restrict(const RestrictArgs A) {
  using SH = Shape<D, TS, 0>;
  constexpr int NIN = TS + 2;
  constexpr int INSZ = ipow(NIN, D);
  constexpr int L0 = SH::size(0);
  constexpr int EPT = L0 / NT;
  constexpr int UP = SH::upper;
  constexpr int KMAX = (SH::max_upper_size + NT - 1) / NT;
  constexpr int PF = (TB * INSZ + NT - 1) / NT;   // prefetched inputs per thread
  constexpr int NCI = 2 * (SH::LTS + 1);          // in-tile channels, li = 2 r + k
  constexpr int NTAP = NCI * (TB + 1);            // staged tap entries per batch
  static_assert(L0 % NT == 0, "tile must be a multiple of the block");
  static_assert(NTAP <= NT, "one thread per staged tap entry");
  __shared__ double s_in[TB * INSZ];
  __shared__ double s_lv[TB * SH::total];
  __shared__ double s_acc[2 * 3 * UP];
  // taps of the in-tile channels for slabs nb-1 .. nb+TB-1: s_q[li][s] is
  // q0 of slab nb-1+s (-1 outside the chunk), s_w[li][s] the weights of
  // slab nb+s
  __shared__ int s_q[NCI][TB + 1];
  __shared__ double s_w[NCI][TB][3];
  __shared__ int s_qlo[NCI];

  const Geometry g = A.g;
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int tx = tile % g.ntile;
  const int ty = (D == 2) ? tile / g.ntile : 0;
  const int chunk = blockIdx.y;
  const int n0 = chunk * g.chunk;
  const int n1 = min(n0 + g.chunk, g.ntf);
  const int ntileD = (D == 2) ? g.ntile * g.ntile : g.ntile;
  const long long nsp = (D == 2) ? (long long)g.nxf * g.nxf : g.nxf;
  const int R = g.R;

  for (int i = tid; i < 2 * 3 * UP; i += NT) s_acc[i] = 0.0;
  if (tid < NCI) {
    const int r = tid >> 1, k = tid & 1;
    int q = 0;
    if (r <= R) {
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (C.active) q = C.q0[n0];
    }
    s_qlo[tid] = q;
  }
  double racc[EPT][2][3];
#pragma unroll
  for (int e = 0; e < EPT; ++e)
#pragma unroll
    for (int k = 0; k < 2; ++k) racc[e][k][0] = racc[e][k][1] = racc[e][k][2] = 0.0;

  // partial block of in-tile channel li at level offset r, time index q
  auto part_index = [&](int li, int r, int q) -> long long {
    const Channel &C = A.ch[(g.J - r - 1) * 2 + (li & 1)];
    return C.part_off +
           (((long long)chunk * ntileD + tile) * C.qb + (q - s_qlo[li])) * (long long)SH::size(r);
  };

  // tap entry staged by this thread: channel li = tid / (TB+1), slab offset
  // my_s; its table pointers are resolved once (independent loads per batch)
  const int my_s = tid % (TB + 1);
  const int *my_q0 = nullptr;
  const double *my_w = nullptr;
  if (tid < NTAP) {
    const int li = tid / (TB + 1), r = li >> 1;
    if (r <= R) {
      const Channel &C = A.ch[(g.J - r - 1) * 2 + (li & 1)];
      if (C.active) {
        my_q0 = C.q0;
        my_w = C.w;
      }
    }
  }
  // register prefetch of one batch (input slabs with halo + tap entries)
  double pin[PF];
  int pq = -1;
  double pw0 = 0.0, pw1 = 0.0, pw2 = 0.0;
  auto fetch = [&](int nb) {
    const int cnt = min(TB, n1 - nb);
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int idx = tid + e * NT;
      double v = 0.0;
      if (idx < cnt * INSZ) {
        const int s = idx / INSZ, loc = idx - s * INSZ;
        const int ix = loc % NIN, iy = loc / NIN;
        const int px = TS * tx - 1 + ix;
        const int py = TS * ty - 1 + iy;
        if (interior(px, g.nxf) && (D == 1 || interior(py, g.nxf))) {
          long long off = (long long)(nb + s) * nsp + (px - 1);
          if (D == 2) off += (long long)(py - 1) * g.nxf;
          v = A.X[off];
        }
      }
      pin[e] = v;
    }
    pq = -1;
    pw0 = pw1 = pw2 = 0.0;
    const int n = nb - 1 + my_s;
    if (my_q0 != nullptr && n >= n0 && n < n1) {
      pq = my_q0[n];
      if (my_s > 0) {
        pw0 = my_w[3 * n];
        pw1 = my_w[3 * n + 1];
        pw2 = my_w[3 * n + 2];
      }
    }
  };

  fetch(n0);
  int last_cnt = 0;
  for (int nb = n0; nb < n1; nb += TB) {
    const int cnt = min(TB, n1 - nb);
    last_cnt = cnt;
    // (1) staged batch -> LDS, then start fetching the next batch
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int idx = tid + e * NT;
      if (idx < TB * INSZ) s_in[idx] = pin[e];
    }
    if (tid < NTAP) {
      const int li = tid / (TB + 1), s = tid - li * (TB + 1);
      s_q[li][s] = pq;
      if (s > 0) {
        s_w[li][s - 1][0] = pw0;
        s_w[li][s - 1][1] = pw1;
        s_w[li][s - 1][2] = pw2;
      }
    }
    __syncthreads();
    if (nb + TB < n1) fetch(nb + TB);
    // (2) level 0 (fine nodes, optional mass stencil) and its accumulation
    for (int s = 0; s < cnt; ++s) {
      const double *in = s_in + s * INSZ;
      double val[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int p = tid + e * NT;
        const int ix = p % TS, iy = (D == 2) ? p / TS : 0;
        const int px = TS * tx + ix, py = TS * ty + iy;
        double v = 0.0;
        if (interior(px, g.nxf) && (D == 1 || interior(py, g.nxf))) {
          if (A.stencil) {
            if (D == 1) {
              v = A.sx * (in[ix] + 4.0 * in[ix + 1] + in[ix + 2]);
            } else {
              const double *r0 = in + iy * NIN + ix, *r1 = r0 + NIN, *r2 = r1 + NIN;
              const double c0 = r0[0] + 4.0 * r0[1] + r0[2];
              const double c1 = r1[0] + 4.0 * r1[1] + r1[2];
              const double c2 = r2[0] + 4.0 * r2[1] + r2[2];
              v = A.sy * A.sx * (c0 + 4.0 * c1 + c2);
            }
          } else {
            v = (D == 1) ? in[ix + 1] : in[(iy + 1) * NIN + ix + 1];
          }
        }
        val[e] = v;
        s_lv[s * SH::total + p] = v;
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (!A.ch[(g.J - 1) * 2 + k].active) continue;
        const int q0n = s_q[k][s + 1], qp = s_q[k][s];
        if (qp >= 0 && q0n > qp) {
          const long long base = part_index(k, 0, qp);
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            A.part[base + tid + e * NT] = racc[e][k][0];
            racc[e][k][0] = racc[e][k][1];
            racc[e][k][1] = racc[e][k][2];
            racc[e][k][2] = 0.0;
          }
        }
        const double w0 = s_w[k][s][0], w1 = s_w[k][s][1], w2 = s_w[k][s][2];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          racc[e][k][0] += w0 * val[e];
          racc[e][k][1] += w1 * val[e];
          racc[e][k][2] += w2 * val[e];
        }
      }
    }
    __syncthreads();
    // (3) restriction pyramid r = 1..R (full weighting, partial at tile edges)
    for (int r = 1; r <= R; ++r) {
      const int nr = SH::nodes(r), np = SH::nodes(r - 1), sz = SH::size(r);
      const int lox = tile_lo(TS, tx, r, 0), plox = tile_lo(TS, tx, r - 1, 0);
      const int loy = tile_lo(TS, ty, r, 0), ploy = tile_lo(TS, ty, r - 1, 0);
      for (int idx = tid; idx < cnt * sz; idx += NT) {
        const int s = idx / sz, j = idx - s * sz;
        const int jx = j % nr, jy = (D == 2) ? j / nr : 0;
        const double *src = s_lv + s * SH::total + SH::offset(r - 1);
        double acc = 0.0;
        const int cx = 2 * (lox + jx) - plox;
        if (D == 1) {
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int sx_ = cx + dx;
            if (sx_ >= 0 && sx_ < np) acc += (dx == 0 ? 1.0 : 0.5) * src[sx_];
          }
        } else {
          const int cy = 2 * (loy + jy) - ploy;
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy) {
            const int sy_ = cy + dy;
            if (sy_ < 0 || sy_ >= np) continue;
            double row = 0.0;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              const int sx_ = cx + dx;
              if (sx_ >= 0 && sx_ < np) row += (dx == 0 ? 1.0 : 0.5) * src[sy_ * np + sx_];
            }
            acc += (dy == 0 ? 1.0 : 0.5) * row;
          }
        }
        s_lv[s * SH::total + SH::offset(r) + j] = acc;
      }
      __syncthreads();
    }
    // (4) accumulate levels r >= 1 into their time nodes (ring of 3 slots)
    for (int r = 1; r <= R; ++r) {
      const int sz = SH::size(r);
      const int aoff = SH::offset(r) - SH::size(0);
      for (int k = 0; k < 2; ++k) {
        const int li = 2 * r + k;
        if (!A.ch[(g.J - r - 1) * 2 + k].active) continue;
        double *acc = s_acc + (size_t)k * 3 * UP + aoff;
        for (int s = 0; s < cnt; ++s) {
          const int q0n = s_q[li][s + 1], qp = s_q[li][s];
          if (qp >= 0 && q0n > qp) {
            const long long base = part_index(li, r, qp);
            double *sl = acc + (qp % 3) * UP;
#pragma unroll
            for (int kk = 0; kk < KMAX; ++kk) {
              const int j = tid + kk * NT;
              if (j < sz) {
                A.part[base + j] = sl[j];
                sl[j] = 0.0;
              }
            }
          }
          const double w0 = s_w[li][s][0], w1 = s_w[li][s][1], w2 = s_w[li][s][2];
          double *a0 = acc + (q0n % 3) * UP;
          double *a1 = acc + ((q0n + 1) % 3) * UP;
          double *a2 = acc + ((q0n + 2) % 3) * UP;
          const double *v = s_lv + s * SH::total + SH::offset(r);
#pragma unroll
          for (int kk = 0; kk < KMAX; ++kk) {
            const int j = tid + kk * NT;
            if (j < sz) {
              const double x = v[j];
              a0[j] += w0 * x;
              a1[j] += w1 * x;
              a2[j] += w2 * x;
            }
          }
        }
      }
      if (r == R && g.A0 > 1 && A.coarse != nullptr) {
        for (int idx = tid; idx < cnt * sz; idx += NT) {
          const int s = idx / sz, j = idx - s * sz;
          A.coarse[((long long)tile * g.ntf + nb + s) * sz + j] =
              s_lv[s * SH::total + SH::offset(r) + j];
        }
      }
    }
    __syncthreads();
  }
  // final flush of the open time nodes (s_q still holds the last batch)
  for (int k = 0; k < 2; ++k) {
    const Channel &C = A.ch[(g.J - 1) * 2 + k];
    if (!C.active) continue;
    const int ql = s_q[k][last_cnt];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      if (ql + o >= C.nq) break;
      const long long base = part_index(k, 0, ql + o);
#pragma unroll
      for (int e = 0; e < EPT; ++e) A.part[base + tid + e * NT] = racc[e][k][o];
    }
  }
  for (int r = 1; r <= R; ++r) {
    const int sz = SH::size(r);
    const int aoff = SH::offset(r) - SH::size(0);
    for (int k = 0; k < 2; ++k) {
      const int li = 2 * r + k;
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (!C.active) continue;
      const int ql = s_q[li][last_cnt];
      for (int o = 0; o < 3; ++o) {
        const int q = ql + o;
        if (q >= C.nq) break;
        const long long base = part_index(li, r, q);
        const double *sl = s_acc + (size_t)k * 3 * UP + aoff + (q % 3) * UP;
        for (int kk = 0; kk < KMAX; ++kk) {
          const int j = tid + kk * NT;
          if (j < sz) A.part[base + j] = sl[j];
        }
      }
    }
  }
}

// Tile range of the tiles whose restriction block holds node P of level
// offset r (blocks [t s_r, t s_r + s_r], s_r = TS >> r; level 0 not shared).
__device__ __forceinline__ void tile_range(int TS, int r, int P, int ntile, int &t0,
                                           int &t1) {
  if (r == 0) {
    t0 = t1 = P / TS;
  } else {
    const int sr = TS >> r;
    t0 = (P + sr - 1) / sr - 1;
    t1 = P / sr;
  }
  if (t0 < 0) t0 = 0;
  if (t1 > ntile - 1) t1 = ntile - 1;
}

template <int D, int TS>
__global__ void k_reduce(const Geometry g, const Channel *__restrict__ ch,
                         const double *__restrict__ part,
                         const WorkItem *__restrict__ items, int nitems,
                         long long total) {
  using SH = Shape<D, TS, 0>;
  const long long gid = gid64();
  if (gid >= total) return;
  int it = 0;
  while (it + 1 < nitems && items[it + 1].start <= gid) ++it;
  const Channel &C = ch[items[it].ch];
  const long long loc = gid - items[it].start;
  const int a = C.a, r = g.J - a;
  const int na = (1 << a) - 1;
  const long long nsp = (D == 2) ? (long long)na * na : na;
  const int q = (int)(loc / nsp);
  const long long K = loc - (long long)q * nsp;
  const int Px = (int)(K % na) + 1;
  const int Py = (D == 2) ? (int)(K / na) + 1 : 0;
  const int nr = SH::nodes(r), sz = SH::size(r);
  const int ntileD = (D == 2) ? g.ntile * g.ntile : g.ntile;
  int tx0, tx1, ty0 = 0, ty1 = 0;
  tile_range(TS, r, Px, g.ntile, tx0, tx1);
  if (D == 2) tile_range(TS, r, Py, g.ntile, ty0, ty1);
  double acc = 0.0;
  for (int c = 0; c < g.nchunk; ++c) {
    const int cn0 = c * g.chunk;
    const int cn1 = min(cn0 + g.chunk, g.ntf);
    const int qlo = C.q0[cn0], qhi = C.q0[cn1 - 1] + 2;
    if (q < qlo || q > qhi) continue;
    for (int ty = ty0; ty <= ty1; ++ty) {
      const int jy = (D == 2) ? Py - tile_lo(TS, ty, r, 0) : 0;
      if (jy < 0 || jy >= nr) continue;
      for (int tx = tx0; tx <= tx1; ++tx) {
        const int jx = Px - tile_lo(TS, tx, r, 0);
        if (jx < 0 || jx >= nr) continue;
        const int tile = ty * g.ntile + tx;
        acc += part[C.part_off +
                    (((long long)c * ntileD + tile) * C.qb + (q - qlo)) * (long long)sz +
                    jy * nr + jx];
      }
    }
  }
  C.data[loc] = C.scale * acc;
}

// S0[n][K0] at the interior nodes of level A0 from the per-slab tile partials
// (each level-A0 node is shared by the tiles t = P-1 and t = P per axis).
template <int D>
__global__ void k_coarse_assemble(const Geometry g, const double *__restrict__ cp,
                                  double *__restrict__ S0) {
  const int na = (1 << g.A0) - 1;
  const long long nsp = (D == 2) ? (long long)na * na : na;
  const long long gid = gid64();
  if (gid >= nsp * g.ntf) return;
  const int n = (int)(gid / nsp);
  const long long K = gid - (long long)n * nsp;
  const int Px = (int)(K % na) + 1;
  const int Py = (D == 2) ? (int)(K / na) + 1 : 0;
  constexpr int SZ = (D == 2) ? 4 : 2;
  double acc = 0.0;
  for (int ty = (D == 2 ? Py - 1 : 0); ty <= (D == 2 ? Py : 0); ++ty) {
    if (ty < 0 || ty >= g.ntile) continue;
    for (int tx = Px - 1; tx <= Px; ++tx) {
      if (tx < 0 || tx >= g.ntile) continue;
      const int tile = (D == 2) ? ty * g.ntile + tx : tx;
      const int j = (D == 2) ? (Py - ty) * 2 + (Px - tx) : (Px - tx);
      acc += cp[((long long)tile * g.ntf + n) * SZ + j];
    }
  }
  S0[gid] = acc;
}

// first index n with q0[n] >= v (q0 nondecreasing)
__device__ __forceinline__ int lower_bound_q(const int *q0, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (q0[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Channels of the levels a < A0: gather over the slabs that touch time node q
// and over the level-A0 nodes in the support of the level-a hat.
template <int D>
__global__ void k_coarse_restrict(const Geometry g, const Channel *__restrict__ ch,
                                  const double *__restrict__ S0,
                                  const WorkItem *__restrict__ items, int nitems,
                                  long long total) {
  const long long gid = gid64();
  if (gid >= total) return;
  int it = 0;
  while (it + 1 < nitems && items[it + 1].start <= gid) ++it;
  const Channel &C = ch[items[it].ch];
  const long long loc = gid - items[it].start;
  const int a = C.a;
  const int na = (1 << a) - 1;
  const long long nsp = (D == 2) ? (long long)na * na : na;
  const int q = (int)(loc / nsp);
  const long long K = loc - (long long)q * nsp;
  const int Px = (int)(K % na) + 1;
  const int Py = (D == 2) ? (int)(K / na) + 1 : 0;
  const int f = 1 << (g.A0 - a);
  const int n0a = (1 << g.A0) - 1;
  const long long nsp0 = (D == 2) ? (long long)n0a * n0a : n0a;
  const int nlo = lower_bound_q(C.q0, g.ntf, q - 2);
  const int nhi = lower_bound_q(C.q0, g.ntf, q + 1);  // exclusive
  double acc = 0.0;
  for (int n = nlo; n < nhi; ++n) {
    const int k = q - C.q0[n];
    if (k < 0 || k > 2) continue;
    const double wq = C.w[3 * n + k];
    if (wq == 0.0) continue;
    const double *S = S0 + (long long)n * nsp0;
    double val = 0.0;
    for (int y = (D == 2 ? (Py - 1) * f + 1 : 0); y <= (D == 2 ? (Py + 1) * f - 1 : 0); ++y) {
      const double wy = (D == 2) ? 1.0 - (double)abs(y - Py * f) / f : 1.0;
      double row = 0.0;
      for (int x = (Px - 1) * f + 1; x <= (Px + 1) * f - 1; ++x) {
        const double wx = 1.0 - (double)abs(x - Px * f) / f;
        row += wx * S[(D == 2 ? (long long)(y - 1) * n0a : 0) + (x - 1)];
      }
      val += wy * row;
    }
    acc += wq * val;
  }
  C.data[loc] = C.scale * acc;
}

// ---------------------------------------------------------- prolongation ---

// C[n][K0] at the interior level-A0 nodes: sum over the channels of levels
// a < A0 of their time-evaluated, linearly interpolated values.
template <int D>
__global__ void k_prolong_coarse(const Geometry g, const Channel *__restrict__ ch,
                                 double *__restrict__ Cout) {
  const int n0a = (1 << g.A0) - 1;
  const long long nsp0 = (D == 2) ? (long long)n0a * n0a : n0a;
  const long long gid = gid64();
  if (gid >= nsp0 * g.ntf) return;
  const int n = (int)(gid / nsp0);
  const long long K0 = gid - (long long)n * nsp0;
  const int P0x = (int)(K0 % n0a) + 1;
  const int P0y = (D == 2) ? (int)(K0 / n0a) + 1 : 0;
  double acc = 0.0;
  for (int a = 1; a < g.A0; ++a) {
    const int f = 1 << (g.A0 - a);
    const int na = (1 << a) - 1;
    const int Lx = P0x / f, rx = P0x - Lx * f;
    const double fx = (double)rx / f;
    const int Ly = (D == 2) ? P0y / f : 0, ry = (D == 2) ? P0y - Ly * f : 0;
    const double fy = (double)ry / f;
    for (int k = 0; k < 2; ++k) {
      const Channel &C = ch[(a - 1) * 2 + k];
      if (!C.active) continue;
      const int q0n = C.q0[n];
      const long long nsp = (D == 2) ? (long long)na * na : na;
      double v = 0.0;
      for (int kk = 0; kk < 3; ++kk) {
        const double w = C.w[3 * n + kk];
        if (w == 0.0) continue;
        const double *Y = C.data + (long long)(q0n + kk) * nsp;
        double s = 0.0;
        for (int oy = 0; oy < (D == 2 ? 2 : 1); ++oy) {
          const int yy = Ly + oy;
          const double wy = (D == 2) ? (oy == 0 ? 1.0 - fy : fy) : 1.0;
          if (wy == 0.0) continue;
          if (D == 2 && !interior(yy, na)) continue;
          for (int ox = 0; ox < 2; ++ox) {
            const int xx = Lx + ox;
            const double wx = ox == 0 ? 1.0 - fx : fx;
            if (wx == 0.0 || !interior(xx, na)) continue;
            s += wy * wx * Y[(D == 2 ? (long long)(yy - 1) * na : 0) + (xx - 1)];
          }
        }
        v += w * s;
      }
      acc += C.scale * v;
    }
  }
  Cout[gid] = acc;
}

template <int D, int TS, int TB, int NT, int MODE>
__global__ void __launch_bounds__(NT) k_prolong(const ProlongArgs A) {
  using SH = Shape<D, TS, MODE>;
  constexpr int L0 = SH::size(0);
  constexpr int EPT0 = (L0 + NT - 1) / NT;
  constexpr int UP = SH::upper;
  constexpr int KMAX = (SH::max_upper_size + NT - 1) / NT;
  constexpr int NO = ipow(TS, D);          // output points per slab
  constexpr int EPTO = NO / NT;
  constexpr int NF = TS + 2 * MODE;
  constexpr int RS = TB + 2;               // coefficient ring slots per channel
  constexpr int NCI = 2 * (SH::LTS + 1);   // in-tile channels, li = 2 r + k
  constexpr int NTAP = NCI * (TB + 1);
  static_assert(NO % NT == 0, "tile must be a multiple of the block");
  static_assert(NTAP <= NT, "one thread per staged tap entry");
  __shared__ double s_v[TB * UP];
  __shared__ double s_coef[2 * RS * UP];
  __shared__ double s_f[MODE ? TB * L0 : 1];
  __shared__ int s_q[NCI][TB + 1];         // q0 of slabs nb-1 .. nb+TB-1 (-1: none)
  __shared__ double s_w[NCI][TB][3];       // weights of slabs nb .. nb+TB-1
  // coarse-level values (levels a < A0, already summed) at the in-tile
  // level-A0 nodes of the batch; used only when A0 > 1, and then R = LTS
  constexpr int SZR = SH::size(SH::LTS);
  static_assert(NTAP + TB * SZR <= NT, "coarse staging threads follow the tap threads");
  __shared__ double s_co[TB * SZR];

  const Geometry g = A.g;
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int tx = tile % g.ntile;
  const int ty = (D == 2) ? tile / g.ntile : 0;
  const int chunk = blockIdx.y;
  const int n0 = chunk * g.chunk;
  const int n1 = min(n0 + g.chunk, g.ntf);
  const long long nsp = (D == 2) ? (long long)g.nxf * g.nxf : g.nxf;
  const int R = g.R;

  // coefficient of channel C at time index q for the node with global
  // positions (Px, Py) of its level (zero outside the interior)
  auto coef = [&](const Channel &C, int q, int Px, int Py) -> double {
    const int na = (1 << C.a) - 1;
    if (!interior(Px, na) || (D == 2 && !interior(Py, na))) return 0.0;
    const long long nspa = (D == 2) ? (long long)na * na : na;
    return C.data[(long long)q * nspa + (D == 2 ? (long long)(Py - 1) * na : 0) + (Px - 1)];
  };

  double rc[EPT0][2][3];  // level-0 coefficient window (q0, q0+1, q0+2)
#pragma unroll
  for (int e = 0; e < EPT0; ++e)
#pragma unroll
    for (int k = 0; k < 2; ++k) rc[e][k][0] = rc[e][k][1] = rc[e][k][2] = 0.0;
  double basev[EPT0];
  const int lo0x = tile_lo(TS, tx, 0, MODE), lo0y = tile_lo(TS, ty, 0, MODE);
#pragma unroll
  for (int e = 0; e < EPT0; ++e) {
    basev[e] = 0.0;
    const int p = tid + e * NT;
    if (!MODE && p < L0 && A.base != nullptr) {
      const int Px = lo0x + p % NF, Py = (D == 2) ? lo0y + p / NF : 0;
      if (interior(Px, g.nxf) && (D == 1 || interior(Py, g.nxf)))
        basev[e] = A.base[(D == 2 ? (long long)(Py - 1) * g.nxf : 0) + (Px - 1)];
    }
  }

  // tap entry staged by this thread (see k_restrict)
  const int my_s = tid % (TB + 1);
  const int *my_q0 = nullptr;
  const double *my_w = nullptr;
  if (tid < NTAP) {
    const int li = tid / (TB + 1), r = li >> 1;
    if (r <= R) {
      const Channel &C = A.ch[(g.J - r - 1) * 2 + (li & 1)];
      if (C.active) {
        my_q0 = C.q0;
        my_w = C.w;
      }
    }
  }
  // tap entries and coarse values of the next batch, prefetched in registers
  int pq = -1;
  double pw0 = 0.0, pw1 = 0.0, pw2 = 0.0, pco = 0.0;
  const bool use_coarse = g.A0 > 1 && A.coarse != nullptr;
  const int co_i = tid - NTAP;  // coarse entry staged by this thread (if >= 0)
  auto fetch_taps = [&](int nb) {
    pq = -1;
    pw0 = pw1 = pw2 = 0.0;
    const int n = nb - 1 + my_s;
    if (my_q0 != nullptr && n >= n0 && n < n1) {
      pq = my_q0[n];
      if (my_s > 0) {
        pw0 = my_w[3 * n];
        pw1 = my_w[3 * n + 1];
        pw2 = my_w[3 * n + 2];
      }
    }
    pco = 0.0;
    if (use_coarse && co_i >= 0 && co_i < TB * SZR) {
      const int s = co_i / SZR, j = co_i - s * SZR;
      constexpr int nrR = SH::nodes(SH::LTS);
      const int Px = tile_lo(TS, tx, SH::LTS, MODE) + j % nrR;
      const int Py = (D == 2) ? tile_lo(TS, ty, SH::LTS, MODE) + j / nrR : 0;
      const int n0a = (1 << g.A0) - 1;
      if (nb + s < n1 && interior(Px, n0a) && (D == 1 || interior(Py, n0a))) {
        const long long nsp0 = (D == 2) ? (long long)n0a * n0a : n0a;
        pco = A.coarse[(long long)(nb + s) * nsp0 +
                       (D == 2 ? (long long)(Py - 1) * n0a : 0) + (Px - 1)];
      }
    }
  };
  // level-J channels belong to time level b = 1 (q0 = 0 on every slab), so
  // their coefficient window is loaded once
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const Channel &C = A.ch[(g.J - 1) * 2 + k];
    if (!C.active) continue;
#pragma unroll
    for (int e = 0; e < EPT0; ++e) {
      const int p = tid + e * NT;
      if (p >= L0) continue;
      const int Px = lo0x + p % NF, Py = (D == 2) ? lo0y + p / NF : 0;
      rc[e][k][0] = coef(C, 0, Px, Py);
      rc[e][k][1] = coef(C, 1, Px, Py);
      rc[e][k][2] = coef(C, 2, Px, Py);
    }
  }

  fetch_taps(n0);
  for (int nb = n0; nb < n1; nb += TB) {
    const int cnt = min(TB, n1 - nb);
    if (tid < NTAP) {
      const int li = tid / (TB + 1), s = tid - li * (TB + 1);
      s_q[li][s] = pq;
      if (s > 0) {
        s_w[li][s - 1][0] = pw0;
        s_w[li][s - 1][1] = pw1;
        s_w[li][s - 1][2] = pw2;
      }
    } else if (co_i < TB * SZR) {
      s_co[co_i] = pco;
    }
    __syncthreads();
    if (nb + TB < n1) fetch_taps(nb + TB);
    // phase A: owners evaluate every level r >= 1 in time.  The coefficients
    // a batch needs beyond those already in the ring are gathered first (all
    // loads of one level in flight together), then the slabs are evaluated.
    for (int r = 1; r <= R; ++r) {
      const int nr = SH::nodes(r), sz = SH::size(r);
      const int aoff = SH::offset(r) - SH::size(0);
      const int lox = tile_lo(TS, tx, r, MODE), loy = tile_lo(TS, ty, r, MODE);
      for (int s = 0; s < cnt; ++s)
#pragma unroll
        for (int kk = 0; kk < KMAX; ++kk) {
          const int j = tid + kk * NT;
          if (j < sz) s_v[s * UP + aoff + j] = 0.0;
        }
      for (int k = 0; k < 2; ++k) {
        const int li = 2 * r + k;
        const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
        if (!C.active) continue;
        double *ring = s_coef + (size_t)k * RS * UP + aoff;
        const int qhi = s_q[li][cnt] + 2;
        const int qnew = s_q[li][0] >= 0 ? s_q[li][0] + 3 : s_q[li][1];
        double cv[RS][KMAX];
#pragma unroll
        for (int o = 0; o < RS; ++o)
#pragma unroll
          for (int kk = 0; kk < KMAX; ++kk) {
            const int j = tid + kk * NT, q = qnew + o;
            cv[o][kk] = (q <= qhi && j < sz)
                            ? coef(C, q, lox + j % nr, (D == 2) ? loy + j / nr : 0)
                            : 0.0;
          }
#pragma unroll
        for (int o = 0; o < RS; ++o)
#pragma unroll
          for (int kk = 0; kk < KMAX; ++kk) {
            const int j = tid + kk * NT, q = qnew + o;
            if (q <= qhi && j < sz) ring[(q % RS) * UP + j] = cv[o][kk];
          }
        for (int s = 0; s < cnt; ++s) {
          const int q0n = s_q[li][s + 1];
          const double w0 = s_w[li][s][0], w1 = s_w[li][s][1], w2 = s_w[li][s][2];
          const double *c0 = ring + (q0n % RS) * UP;
          const double *c1 = ring + ((q0n + 1) % RS) * UP;
          const double *c2 = ring + ((q0n + 2) % RS) * UP;
#pragma unroll
          for (int kk = 0; kk < KMAX; ++kk) {
            const int j = tid + kk * NT;
            if (j < sz) s_v[s * UP + aoff + j] += C.scale * (w0 * c0[j] + w1 * c1[j] + w2 * c2[j]);
          }
        }
      }
    }
    __syncthreads();
    // phase B: top-down interpolation r = R .. 1 (values of level r+1 are final)
    for (int r = R; r >= 1; --r) {
      const int nr = SH::nodes(r), sz = SH::size(r);
      const int aoff = SH::offset(r) - SH::size(0);
      const int lox = tile_lo(TS, tx, r, MODE), loy = tile_lo(TS, ty, r, MODE);
      for (int idx = tid; idx < cnt * sz; idx += NT) {
        const int s = idx / sz, j = idx - s * sz;
        const int Px = lox + j % nr, Py = (D == 2) ? loy + j / nr : 0;
        double base = 0.0;
        if (r == R) {
          if (use_coarse) base = s_co[s * SZR + j];
        } else {
          const int pn = SH::nodes(r + 1);
          const int paoff = SH::offset(r + 1) - SH::size(0);
          const int plox = tile_lo(TS, tx, r + 1, MODE), ploy = tile_lo(TS, ty, r + 1, MODE);
          const double *par = s_v + s * UP + paoff;
          const int xl = (Px >> 1) - plox, xh = ((Px + 1) >> 1) - plox;
          if (D == 1) {
            base = 0.5 * (par[xl] + par[xh]);
          } else {
            const int yl = (Py >> 1) - ploy, yh = ((Py + 1) >> 1) - ploy;
            base = 0.25 * (par[yl * pn + xl] + par[yl * pn + xh] + par[yh * pn + xl] +
                           par[yh * pn + xh]);
          }
        }
        s_v[s * UP + aoff + j] += base;
      }
      __syncthreads();
    }
    // phase C: fine nodes (owners, slabs in order for the register window)
    for (int s = 0; s < cnt; ++s) {
      const int n = nb + s;
      double tv[EPT0];
#pragma unroll
      for (int e = 0; e < EPT0; ++e) tv[e] = 0.0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const Channel &C = A.ch[(g.J - 1) * 2 + k];
        if (!C.active) continue;
        const double w0 = s_w[k][s][0], w1 = s_w[k][s][1], w2 = s_w[k][s][2];
#pragma unroll
        for (int e = 0; e < EPT0; ++e)
          tv[e] += C.scale * (w0 * rc[e][k][0] + w1 * rc[e][k][1] + w2 * rc[e][k][2]);
      }
#pragma unroll
      for (int e = 0; e < EPT0; ++e) {
        const int p = tid + e * NT;
        if (p >= L0) continue;
        const int Px = lo0x + p % NF, Py = (D == 2) ? lo0y + p / NF : 0;
        double v = tv[e];
        if (R >= 1) {
          const int pn = SH::nodes(1);
          const int plox = tile_lo(TS, tx, 1, MODE), ploy = tile_lo(TS, ty, 1, MODE);
          const double *par = s_v + s * UP;  // level 1 sits at offset 0 of s_v
          const int xl = (Px >> 1) - plox, xh = ((Px + 1) >> 1) - plox;
          if (D == 1) {
            v += 0.5 * (par[xl] + par[xh]);
          } else {
            const int yl = (Py >> 1) - ploy, yh = ((Py + 1) >> 1) - ploy;
            v += 0.25 * (par[yl * pn + xl] + par[yl * pn + xh] + par[yh * pn + xl] +
                         par[yh * pn + xh]);
          }
        }
        const bool in = interior(Px, g.nxf) && (D == 1 || interior(Py, g.nxf));
        if (MODE) {
          s_f[s * L0 + p] = in ? v : 0.0;
        } else if (in) {
          const long long off = (long long)n * nsp +
                                (D == 2 ? (long long)(Py - 1) * g.nxf : 0) + (Px - 1);
          double o = v + basev[e];
          if (A.accumulate) o += A.out[off];
          A.out[off] = o;
        }
      }
    }
    if (MODE) {
      __syncthreads();
      for (int s = 0; s < cnt; ++s) {
        const int n = nb + s;
        const double *f = s_f + s * L0;
#pragma unroll
        for (int e = 0; e < EPTO; ++e) {
          const int p = tid + e * NT;
          const int ix = p % TS, iy = (D == 2) ? p / TS : 0;
          const int Px = TS * tx + ix, Py = (D == 2) ? TS * ty + iy : 0;
          if (!interior(Px, g.nxf) || (D == 2 && !interior(Py, g.nxf))) continue;
          double v;
          if (D == 1) {
            v = A.sx * (f[ix] + 4.0 * f[ix + 1] + f[ix + 2]);
          } else {
            const double *r0 = f + iy * NF + ix, *r1 = r0 + NF, *r2 = r1 + NF;
            v = A.sy * A.sx * ((r0[0] + 4.0 * r0[1] + r0[2]) + 4.0 * (r1[0] + 4.0 * r1[1] + r1[2]) +
                               (r2[0] + 4.0 * r2[1] + r2[2]));
          }
          const long long off = (long long)n * nsp +
                                (D == 2 ? (long long)(Py - 1) * g.nxf : 0) + (Px - 1);
          double base = 0.0;
          if (A.base != nullptr) base = A.base[(D == 2 ? (long long)(Py - 1) * g.nxf : 0) + (Px - 1)];
          double o = v + base;
          if (A.accumulate) o += A.out[off];
          A.out[off] = o;
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- small kernels -----

// Fine-grid mass and stiffness stencils (per-element c^2 on the finest mesh).
//   mode 0: mv = M v,  ku = K u
//   mode 1: mv = M v,  ku = gsum - K u      (adjoint of the lift and u0 term)
template <int D>
__global__ void k_fine_stencils(int N, const double *__restrict__ ce, double hx,
                                double hy, const double *__restrict__ v,
                                const double *__restrict__ u, double *__restrict__ mv,
                                double *__restrict__ ku, const double *__restrict__ gsum,
                                int mode) {
  const int n = N - 1;
  const long long nsp = (D == 2) ? (long long)n * n : n;
  const long long gid = gid64();
  if (gid >= nsp) return;
  const int Px = (int)(gid % n) + 1;
  const int Py = (D == 2) ? (int)(gid / n) + 1 : 0;
  auto at = [&](const double *f, int x, int y) -> double {
    if (!interior(x, n) || (D == 2 && !interior(y, n))) return 0.0;
    return f[(D == 2 ? (long long)(y - 1) * n : 0) + (x - 1)];
  };
  if (mv != nullptr) {
    double r;
    if (D == 1) {
      r = hx / 6.0 * (at(v, Px - 1, 0) + 4.0 * at(v, Px, 0) + at(v, Px + 1, 0));
    } else {
      double rows[3];
      for (int dy = -1; dy <= 1; ++dy)
        rows[dy + 1] = at(v, Px - 1, Py + dy) + 4.0 * at(v, Px, Py + dy) + at(v, Px + 1, Py + dy);
      r = hx / 6.0 * hy / 6.0 * (rows[0] + 4.0 * rows[1] + rows[2]);
    }
    mv[gid] = r;
  }
  if (ku != nullptr) {
    double r = 0.0;
    if (D == 1) {
      const double c2l = ce[Px - 1], c2r = ce[Px];
      const double u0 = at(u, Px, 0);
      r = (c2l * (u0 - at(u, Px - 1, 0)) + c2r * (u0 - at(u, Px + 1, 0))) / hx;
    } else {
      // Q1 element stiffness c^2 (kx (x) my + mx (x) ky) summed over the four
      // elements around the node; element (ey,ex) spans positions ey..ey+1.
      for (int ey = Py - 1; ey <= Py; ++ey)
        for (int ex = Px - 1; ex <= Px; ++ex) {
          const double c2 = ce[(long long)ey * N + ex];
          const int ly = Py - ey, lx = Px - ex;
          for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
              const double kxv = (lx == cx ? 1.0 : -1.0) / hx;
              const double mxv = hx / 6.0 * (lx == cx ? 2.0 : 1.0);
              const double kyv = (ly == cy ? 1.0 : -1.0) / hy;
              const double myv = hy / 6.0 * (ly == cy ? 2.0 : 1.0);
              r += c2 * (kxv * myv + mxv * kyv) * at(u, ex + cx, ey + cy);
            }
        }
    }
    ku[gid] = (mode == 1) ? gsum[gid] - r : r;
  }
}

__device__ __forceinline__ int find_comp(const CompDesc *cd, int ncomp, long long gid) {
  int c = 0;
  while (c + 1 < ncomp && cd[c + 1].start <= gid) ++c;
  return c;
}

// b_c[i][K] = sum_q D_b[i][q] Z_c[q][K] + psi_i'(0) MV_a[K] - g_b[i] KU_a[K]
__global__ void k_post_load(const CompDesc *__restrict__ cd, int ncomp, long long total,
                            const KernelTables *__restrict__ kt) {
  const long long gid = gid64();
  if (gid >= total) return;
  const CompDesc &C = cd[find_comp(cd, ncomp, gid)];
  const long long loc = gid - C.start;
  const int i = (int)(loc / C.nsp);
  const long long K = loc - (long long)i * C.nsp;
  const double *Z = C.z;
  double v = kt->Dlo[C.b][i] * Z[loc];
  if (i + 1 < C.nq) v += kt->Dhi[C.b][i] * Z[loc + C.nsp];
  if (i == 0 && C.mv != nullptr) v += kt->Dlo[C.b][0] * C.mv[K];
  if (C.ku != nullptr) v -= kt->g[C.b][i] * C.ku[K];
  C.data[loc] = v;
}

// zeta_c[q][K] = sum_i D_b[i][q] z_c[i][K]   (transpose of the above)
__global__ void k_post_adjoint(const CompDesc *__restrict__ cd, int ncomp,
                               long long total, const KernelTables *__restrict__ kt) {
  const long long gid = gid64();
  if (gid >= total) return;
  const CompDesc &C = cd[find_comp(cd, ncomp, gid)];
  const long long loc = gid - C.start;
  const int q = (int)(loc / C.nsp);
  double v = kt->Dlo[C.b][q] * C.z[loc];
  if (q >= 1) v += kt->Dhi[C.b][q - 1] * C.z[loc - C.nsp];
  C.data[loc] = v;
}

// fv_a[K] = sum_c psi_0'(0) z_c[0][K];  fu_a[K] = sum_c sum_i g_b[i] z_c[i][K]
__global__ void k_adjoint_fields(const LevelDesc *__restrict__ ld, int nlev,
                                 long long total, const CompDesc *__restrict__ cd,
                                 const KernelTables *__restrict__ kt) {
  const long long gid = gid64();
  if (gid >= total) return;
  int l = 0;
  while (l + 1 < nlev && ld[l + 1].start <= gid) ++l;
  const LevelDesc &L = ld[l];
  const long long K = gid - L.start;
  double fv = 0.0, fu = 0.0;
  for (int t = 0; t < 2; ++t) {
    const int c = t == 0 ? L.c0 : L.c1;
    if (c < 0) continue;
    const CompDesc &C = cd[c];
    fv += kt->Dlo[C.b][0] * C.z[K];
    const double *gb = kt->g[C.b];
    double s = 0.0;
    for (int i = 0; i < C.nq; ++i) s += gb[i] * C.z[(long long)i * C.nsp + K];
    fu += s;
  }
  L.fv[K] = fv;
  L.fu[K] = fu;
}

// Batched C = A B (row major), 64x64 tiles, 256 threads, 4x4 outputs each.
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc *__restrict__ descs,
                                              int ndesc) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  int di = 0;
  while (di + 1 < ndesc && descs[di + 1].tile0 <= (int)blockIdx.x) ++di;
  const GemmDesc &Dd = descs[di];
  int t = blockIdx.x - Dd.tile0;
  const int per = Dd.tm * Dd.tn;
  const int bidx = t / per;
  t -= bidx * per;
  const int tmi = t / Dd.tn, tni = t - tmi * Dd.tn;
  const double *Ap = Dd.A + bidx * Dd.sA;
  const double *Bp = Dd.B + bidx * Dd.sB;
  double *Cp = Dd.C + bidx * Dd.sC;
  const int row0 = tmi * BM, col0 = tni * BN;
  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < Dd.K; k0 += BK) {
    for (int i = tid; i < BM * BK; i += 256) {
      const int m = i / BK, k = i % BK;
      const int gm = row0 + m, gk = k0 + k;
      As[k][m] = (gm < Dd.M && gk < Dd.K) ? Ap[(long long)gm * Dd.lda + gk] : 0.0;
    }
    for (int i = tid; i < BK * BN; i += 256) {
      const int k = i / BN, nn = i % BN;
      const int gk = k0 + k, gn = col0 + nn;
      Bs[k][nn] = (gk < Dd.K && gn < Dd.N) ? Bp[(long long)gk * Dd.ldb + gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[k][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[k][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = row0 + ty * 4 + i;
    if (gm >= Dd.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = col0 + tx * 4 + j;
      if (gn < Dd.N) Cp[(long long)gm * Dd.ldc + gn] = acc[i][j];
    }
  }
}

// ---- per-mode banded time solve ------------------------------------------

// Double-double helpers.  Floating-point contraction must stay off inside
// them: a product p = a*b fused with a later subtraction (acc - p) into one
// FMA uses the unrounded product while the error term assumes the rounded
// one, which silently destroys the error-free transformation.
struct dd {
  double h, l;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
  dd s = two_sum(x.h, y.h);
  s.l += x.l + y.l;
  return two_sum(s.h, s.l);
}
// (p * q) * x with p, q, x doubles, as a double-double
__device__ __forceinline__ dd triple(double p, double q, double x) {
#pragma clang fp contract(off)
  const dd pq = two_prod(p, q);
  dd r = two_prod(pq.h, x);
  r.l = fma(pq.l, x, r.l);
  return r;
}

// One thread per spatial mode: (m A_b + kappa B_b) u = r, or its transpose.
// E = m A_b + kappa B_b is factored E = L U without pivoting in causal
// (increasing time) order - the symmetric parts of A_b and B_b are positive
// definite (Prop. 1).  The factors depend only on (m, kappa, b) and are
// computed once when the plan is built.  The transposed (adjoint) system uses
// the same factors, E^T = U^T L^T, which keeps the elimination causal for the
// backward-in-time adjoint.  The solution is refined against the
// double-double time matrices.
//
// Every descriptor starts at a multiple of 64 threads and blocks are one wave,
// so the descriptor, its tables and the time level are wave-uniform.

__device__ __forceinline__ int find_solve(const SolveDesc *sds, int nsd, long long wbase) {
  int lo = 0, hi = nsd - 1;  // last descriptor with thread0 <= wbase
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sds[mid].thread0 <= wbase) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void mode_scalars(const SolveDesc &S, int j,
                                             const ModeTables *mt, int d, double &m,
                                             double &kap) {
  const int a = S.a, na = (1 << a) - 1;
  if (d == 1) {
    m = mt->mx[a][j];
    kap = S.c2 * mt->kx[a][j];
  } else {
    const int jx = j % na, jy = j / na;
    m = mt->my[a][jy] * mt->mx[a][jx];
    kap = S.c2 * (mt->ky[a][jy] * mt->mx[a][jx] + mt->my[a][jy] * mt->kx[a][jx]);
  }
}

__global__ void __launch_bounds__(64) k_time_factor(const SolveDesc *__restrict__ sds,
                                                    int nsd, long long total,
                                                    const KernelTables *__restrict__ kt,
                                                    const ModeTables *__restrict__ mt, int d) {
  const long long wbase = (long long)blockIdx.x * 64;
  const SolveDesc &S = sds[find_solve(sds, nsd, wbase)];
  const long long gid = wbase + threadIdx.x;
  const int j = (int)(gid - S.thread0);
  if (gid >= total || j >= S.nmodes) return;
  const int b = S.b, nq = S.nq, nm = S.nmodes;
  double m, kap;
  mode_scalars(S, j, mt, d, m, kap);
  const double *Ab = kt->A[b], *Bb = kt->B[b];
  auto ent = [&](int i, int off) -> double {
    const int jj = i + off;
    if (jj < 0 || jj >= nq) return 0.0;
    return m * Ab[i * 5 + off + 2] + kap * Bb[i * 5 + off + 2];
  };
  const long long plane = (long long)nq * nm;
  double *L1 = S.fac, *L2 = L1 + plane, *UD = L2 + plane, *U1 = UD + plane, *U2 = U1 + plane;
  double dm2 = 1.0, u1m2 = 0.0, u2m2 = 0.0;
  double dm1 = 1.0, u1m1 = 0.0, u2m1 = 0.0;
  for (int i = 0; i < nq; ++i) {
    const long long o = (long long)i * nm + j;
    double am2 = ent(i, -2), am1 = ent(i, -1), a0 = ent(i, 0), ap1 = ent(i, 1),
           ap2 = ent(i, 2);
    const double l2 = (i >= 2) ? am2 / dm2 : 0.0;
    am1 -= l2 * u1m2;
    a0 -= l2 * u2m2;
    const double l1 = (i >= 1) ? am1 / dm1 : 0.0;
    a0 -= l1 * u1m1;
    ap1 -= l1 * u2m1;
    L1[o] = l1;
    L2[o] = l2;
    UD[o] = 1.0 / a0;
    U1[o] = ap1;
    U2[o] = ap2;
    dm2 = dm1; u1m2 = u1m1; u2m2 = u2m1;
    dm1 = a0; u1m1 = ap1; u2m1 = ap2;
  }
}

__global__ void __launch_bounds__(64) k_time_solve(const SolveDesc *__restrict__ sds,
                                                   int nsd, long long total,
                                                   const KernelTables *__restrict__ kt,
                                                   const ModeTables *__restrict__ mt, int d) {
  constexpr int CH = 16;  // rows per register chunk of a substitution
  constexpr int CR = 8;   // rows per register chunk of the residual
  const long long wbase = (long long)blockIdx.x * 64;
  const SolveDesc &S = sds[find_solve(sds, nsd, wbase)];
  const long long gid = wbase + threadIdx.x;
  const int j = (int)(gid - S.thread0);
  if (gid >= total || j >= S.nmodes) return;
  const int b = S.b, nq = S.nq, nm = S.nmodes;
  double m, kap;
  mode_scalars(S, j, mt, d, m, kap);
  const double *Ab = kt->A[b], *Bb = kt->B[b], *Al = kt->Alo[b], *Bl = kt->Blo[b];
  const bool tr = S.transpose != 0;
  double *rhs = S.rhs;
  const long long plane = (long long)nq * nm;
  const double *L1 = S.fac, *L2 = L1 + plane, *UD = L2 + plane, *U1 = UD + plane,
               *U2 = U1 + plane;
  double *Y = S.scratch, *B0 = Y + plane;
  auto idx = [&](int i) -> long long { return (long long)i * nm + j; };

  // x <- op(E)^{-1} r, r read from R (R may be Y: a chunk is read before it is
  // written), result added to (add) or stored into rhs; returns max |x|
  auto apply_inverse = [&](const double *R, bool add) -> double {
    double xm = 0.0;
    if (!tr) {
      // L y = r (forward)
      double ym2 = 0.0, ym1 = 0.0;
      for (int i0 = 0; i0 < nq; i0 += CH) {
        double rr[CH], l1[CH], l2[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i0 + k;
          if (i < nq) {
            rr[k] = R[idx(i)];
            l1[k] = L1[idx(i)];
            l2[k] = L2[idx(i)];
          }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i0 + k;
          if (i < nq) {
            const double y = rr[k] - l2[k] * ym2 - l1[k] * ym1;
            Y[idx(i)] = y;
            ym2 = ym1;
            ym1 = y;
          }
        }
      }
      // U x = y (backward)
      double xp1 = 0.0, xp2 = 0.0;
      for (int i1 = nq - 1; i1 >= 0; i1 -= CH) {
        double yy[CH], u1[CH], u2[CH], ud[CH], old[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i1 - k;
          if (i >= 0) {
            yy[k] = Y[idx(i)];
            u1[k] = U1[idx(i)];
            u2[k] = U2[idx(i)];
            ud[k] = UD[idx(i)];
            old[k] = add ? rhs[idx(i)] : 0.0;
          }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i1 - k;
          if (i >= 0) {
            const double x = (yy[k] - u1[k] * xp1 - u2[k] * xp2) * ud[k];
            rhs[idx(i)] = add ? old[k] + x : x;
            xm = fmax(xm, fabs(x));
            xp2 = xp1;
            xp1 = x;
          }
        }
      }
    } else {
      // U^T w = r (forward)
      double wm2 = 0.0, wm1 = 0.0;
      for (int i0 = 0; i0 < nq; i0 += CH) {
        double rr[CH], u1[CH], u2[CH], ud[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i0 + k;
          if (i < nq) {
            rr[k] = R[idx(i)];
            u1[k] = i >= 1 ? U1[idx(i - 1)] : 0.0;
            u2[k] = i >= 2 ? U2[idx(i - 2)] : 0.0;
            ud[k] = UD[idx(i)];
          }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i0 + k;
          if (i < nq) {
            const double w = (rr[k] - u1[k] * wm1 - u2[k] * wm2) * ud[k];
            Y[idx(i)] = w;
            wm2 = wm1;
            wm1 = w;
          }
        }
      }
      // L^T z = w (backward)
      double zp1 = 0.0, zp2 = 0.0;
      for (int i1 = nq - 1; i1 >= 0; i1 -= CH) {
        double yy[CH], l1[CH], l2[CH], old[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i1 - k;
          if (i >= 0) {
            yy[k] = Y[idx(i)];
            l1[k] = i + 1 < nq ? L1[idx(i + 1)] : 0.0;
            l2[k] = i + 2 < nq ? L2[idx(i + 2)] : 0.0;
            old[k] = add ? rhs[idx(i)] : 0.0;
          }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = i1 - k;
          if (i >= 0) {
            const double z = yy[k] - l1[k] * zp1 - l2[k] * zp2;
            rhs[idx(i)] = add ? old[k] + z : z;
            xm = fmax(xm, fabs(z));
            zp2 = zp1;
            zp1 = z;
          }
        }
      }
    }
    return xm;
  };
  if (S.refine)
    for (int i = 0; i < nq; ++i) B0[idx(i)] = rhs[idx(i)];
  apply_inverse(rhs, false);
  // refinement: r = b - op(E) x with E from the double-double time matrices,
  // accumulated in double-double, then x += op(E)^{-1} r; stop once the
  // correction is below 1e-15 of the solution (the next one would be below
  // the rounding of x itself)
  for (int it = 0; it < S.refine; ++it) {
#pragma clang fp contract(off)
    double xmax = 0.0;
    for (int i0 = 0; i0 < nq; i0 += CR) {
      double res[CR];
#pragma unroll
      for (int k = 0; k < CR; ++k) {
        const int i = i0 + k;
        if (i >= nq) continue;
        dd acc = {B0[idx(i)], 0.0};
#pragma unroll
        for (int off = -2; off <= 2; ++off) {
          const int jj = i + off;
          if (jj < 0 || jj >= nq) continue;
          // op(E)[i][jj] = E[i][jj] (or E[jj][i] for the transpose)
          const int r = tr ? jj : i, c = tr ? 2 - off : off + 2;
          const double x = rhs[idx(jj)];
          if (off == 0) xmax = fmax(xmax, fabs(x));
          dd t1 = triple(m, Ab[r * 5 + c], x);
          dd t2 = triple(kap, Bb[r * 5 + c], x);
          t1.l = fma(m * Al[r * 5 + c], x, t1.l);
          t2.l = fma(kap * Bl[r * 5 + c], x, t2.l);
          acc = dd_add(acc, {-t1.h, -t1.l});
          acc = dd_add(acc, {-t2.h, -t2.l});
        }
        res[k] = acc.h + acc.l;
      }
#pragma unroll
      for (int k = 0; k < CR; ++k)
        if (i0 + k < nq) Y[idx(i0 + k)] = res[k];
    }
    const double dmax = apply_inverse(Y, true);
    if (dmax <= 1e-15 * xmax) break;
  }
}

__global__ void k_fill(double *p, long long n, double v) {
  const long long i = gid64();
  if (i < n) p[i] = v;
}

__global__ void k_broadcast(double *out, const double *base, int nt, long long nsp) {
  const long long i = gid64();
  if (i < (long long)nt * nsp) out[i] = base != nullptr ? base[i % nsp] : 0.0;
}

// ------------------------------------------------------------ launchers ----

static inline unsigned blocks_for(long long n, int bs) {
  return (unsigned)((n + bs - 1) / bs);
}

constexpr int kTS2 = 32, kTB2 = 2, kTS1 = 256, kTB1 = 8, kNT = 256;

hipError_t launch_restrict(const RestrictArgs &a, hipStream_t s) {
  const int nt = a.g.d == 2 ? a.g.ntile * a.g.ntile : a.g.ntile;
  dim3 grid(nt, a.g.nchunk);
  if (a.g.d == 2)
    hipLaunchKernelGGL((k_restrict<2, kTS2, kTB2, kNT>), grid, dim3(kNT), 0, s, a);
  else
    hipLaunchKernelGGL((k_restrict<1, kTS1, kTB1, kNT>), grid, dim3(kNT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const Geometry &g, const Channel *ch, const double *part,
                         const WorkItem *items, int nitems, long long total,
                         hipStream_t s) {
  if (total == 0) return hipSuccess;
  if (g.d == 2)
    hipLaunchKernelGGL((k_reduce<2, kTS2>), dim3(blocks_for(total, 256)), dim3(256), 0, s,
                       g, ch, part, items, nitems, total);
  else
    hipLaunchKernelGGL((k_reduce<1, kTS1>), dim3(blocks_for(total, 256)), dim3(256), 0, s,
                       g, ch, part, items, nitems, total);
  return hipGetLastError();
}

hipError_t launch_coarse_assemble(const Geometry &g, const double *cp, double *S0,
                                  hipStream_t s) {
  const long long na = (1 << g.A0) - 1;
  const long long n = (g.d == 2 ? na * na : na) * g.ntf;
  if (g.d == 2)
    hipLaunchKernelGGL(k_coarse_assemble<2>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, cp, S0);
  else
    hipLaunchKernelGGL(k_coarse_assemble<1>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, cp, S0);
  return hipGetLastError();
}

hipError_t launch_coarse_restrict(const Geometry &g, const Channel *ch, const double *S0,
                                  const WorkItem *items, int nitems, long long total,
                                  hipStream_t s) {
  if (total == 0) return hipSuccess;
  if (g.d == 2)
    hipLaunchKernelGGL(k_coarse_restrict<2>, dim3(blocks_for(total, 128)), dim3(128), 0, s,
                       g, ch, S0, items, nitems, total);
  else
    hipLaunchKernelGGL(k_coarse_restrict<1>, dim3(blocks_for(total, 128)), dim3(128), 0, s,
                       g, ch, S0, items, nitems, total);
  return hipGetLastError();
}

hipError_t launch_prolong_coarse(const Geometry &g, const Channel *ch, double *C, int,
                                 hipStream_t s) {
  const long long na = (1 << g.A0) - 1;
  const long long n = (g.d == 2 ? na * na : na) * g.ntf;
  if (g.d == 2)
    hipLaunchKernelGGL(k_prolong_coarse<2>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, ch, C);
  else
    hipLaunchKernelGGL(k_prolong_coarse<1>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, ch, C);
  return hipGetLastError();
}

hipError_t launch_prolong(const ProlongArgs &a, hipStream_t s) {
  const int nt = a.g.d == 2 ? a.g.ntile * a.g.ntile : a.g.ntile;
  dim3 grid(nt, a.g.nchunk);
  if (a.g.d == 2) {
    if (a.stencil)
      hipLaunchKernelGGL((k_prolong<2, kTS2, kTB2, kNT, 1>), grid, dim3(kNT), 0, s, a);
    else
      hipLaunchKernelGGL((k_prolong<2, kTS2, kTB2, kNT, 0>), grid, dim3(kNT), 0, s, a);
  } else {
    if (a.stencil)
      hipLaunchKernelGGL((k_prolong<1, kTS1, kTB1, kNT, 1>), grid, dim3(kNT), 0, s, a);
    else
      hipLaunchKernelGGL((k_prolong<1, kTS1, kTB1, kNT, 0>), grid, dim3(kNT), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fine_stencils(int d, int N, const double *ce, double hx, double hy,
                                const double *v_in, const double *u_in, double *mv_out,
                                double *ku_out, const double *gsum, int mode,
                                hipStream_t s) {
  const long long n = N - 1;
  const long long nsp = d == 2 ? n * n : n;
  if (d == 2)
    hipLaunchKernelGGL(k_fine_stencils<2>, dim3(blocks_for(nsp, 256)), dim3(256), 0, s, N, ce,
                       hx, hy, v_in, u_in, mv_out, ku_out, gsum, mode);
  else
    hipLaunchKernelGGL(k_fine_stencils<1>, dim3(blocks_for(nsp, 256)), dim3(256), 0, s, N, ce,
                       hx, hy, v_in, u_in, mv_out, ku_out, gsum, mode);
  return hipGetLastError();
}

hipError_t launch_post_load(const CompDesc *cd, int ncomp, long long total,
                            const KernelTables *kt, hipStream_t s) {
  hipLaunchKernelGGL(k_post_load, dim3(blocks_for(total, 256)), dim3(256), 0, s, cd, ncomp,
                     total, kt);
  return hipGetLastError();
}

hipError_t launch_post_adjoint(const CompDesc *cd, int ncomp, long long total,
                               const KernelTables *kt, hipStream_t s) {
  hipLaunchKernelGGL(k_post_adjoint, dim3(blocks_for(total, 256)), dim3(256), 0, s, cd,
                     ncomp, total, kt);
  return hipGetLastError();
}

hipError_t launch_adjoint_fields(const LevelDesc *ld, int nlev, long long total,
                                 const CompDesc *cd, const KernelTables *kt,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_fields, dim3(blocks_for(total, 256)), dim3(256), 0, s, ld,
                     nlev, total, cd, kt);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmDesc *descs, int ndesc, int total_tiles, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm, dim3(total_tiles), dim3(256), 0, s, descs, ndesc);
  return hipGetLastError();
}

hipError_t launch_time_factor(const SolveDesc *sd, int nsd, long long total,
                              const KernelTables *kt, const ModeTables *mt, int d,
                              hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_factor, dim3(blocks_for(total, 64)), dim3(64), 0, s, sd, nsd,
                     total, kt, mt, d);
  return hipGetLastError();
}

hipError_t launch_time_solve(const SolveDesc *sd, int nsd, long long total,
                             const KernelTables *kt, const ModeTables *mt, int d,
                             hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_solve, dim3(blocks_for(total, 64)), dim3(64), 0, s, sd, nsd,
                     total, kt, mt, d);
  return hipGetLastError();
}

hipError_t launch_fill(double *p, long long n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_broadcast(double *out, const double *base, int nt, long long nsp,
                            hipStream_t s) {
  const long long n = (long long)nt * nsp;
  hipLaunchKernelGGL(k_broadcast, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, base, nt,
                     nsp);
  return hipGetLastError();
}

}  // namespace sg
