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

#include <map>
#include <mutex>

#include "kernels.hpp"
#include "gmem.hpp"
#include "tables.hpp"

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

// linear block index of a 2-D launch grid
__device__ __forceinline__ int block_lin() { return blockIdx.y * gridDim.x + blockIdx.x; }

// first global thread of the calling wave, given its block's first thread
// (wave-uniform)
__device__ __forceinline__ long long wave_gid0(long long block_first) {
  return block_first + __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
}

// --------------------------------------------------------- restriction -----

// XCD-aware block order for the streaming kernels.  Workgroups are dealt
// round-robin to the 8 XCDs (each with its own L2); the logical (chunk, tile)
// of hardware block b is chosen so that every XCD holds a contiguous run of
// tiles of one time chunk, and neighbouring tiles - which read each other's
// halo rows - share an L2.
// lin: the block's linear index in its launch (or, in a launch of many
// problems, in its problem's range of blocks, which starts at a multiple of 8)
__device__ __forceinline__ void stream_block(int lin, int ntileD, int nchunk, int &tile,
                                             int &chunk) {
  const int total = ntileD * nchunk;
  if (total % 8 == 0) lin = (lin & 7) * (total >> 3) + (lin >> 3);
  chunk = lin / ntileD;
  tile = lin - chunk * ntileD;
}

// Zero-halo LDS layout of the in-tile levels (one copy per slab).  Level r
// keeps its nodes(r)^D values at padded index (jy+1)*pn(r) + (jx+1); the halo
// entries stay zero, so the full-weighting stencil of a level-(r+1) node reads
// padded entries (2jy+dy)*pn(r) + 2jx+dx, dx, dy in {0,1,2}, without tests.
// Level 0 gets two halo entries on the far side (its coarse neighbour reaches
// one node past the tile).
template <int D, int TS, int MODE>
struct Pad {
  using SH = Shape<D, TS, MODE>;
  __host__ __device__ static constexpr int pn(int r) { return SH::nodes(r) + (r == 0 ? 3 : 2); }
  __host__ __device__ static constexpr int psize(int r) { return ipow(pn(r), D); }
  __host__ __device__ static constexpr int poff(int r) { return r == 0 ? 0 : poff(r - 1) + psize(r - 1); }
  static constexpr int total = poff(SH::LTS + 1);
};

// Upper-level nodes (levels r = 1..LTS of the tile) are owned by threads:
// thread t owns upper nodes u = t and u = t + NT.  An owned node knows its
// level, its row-major index j in the level and its relative coordinates.
template <int D, int TS, int MODE>
struct Owned {
  int r = 0;  // 0: no node in this slot
  int j = 0, jx = 0, jy = 0;
  __device__ void set(int u) {
    using SH = Shape<D, TS, MODE>;
    r = 0;
    int base = 0;
#pragma unroll
    for (int rr = 1; rr <= SH::LTS; ++rr) {
      const int sz = SH::size(rr);
      if (r == 0 && u >= base && u < base + sz) {
        r = rr;
        j = u - base;
        jx = j % SH::nodes(rr);
        jy = (D == 2) ? j / SH::nodes(rr) : 0;
      }
      base += sz;
    }
  }
};

// Full weighting of a level-(r) node from the padded level r-1 array (PN is
// a constant once the level loop is unrolled).
template <int D>
__device__ __forceinline__ double full_weight(const double *src, int PN, int jx, int jy) {
  if (D == 1) {
    const double *p = src + 2 * jx;
    return 0.5 * (p[0] + p[2]) + p[1];
  } else {
    const double *p = src + 2 * jy * PN + 2 * jx;
    const double r0 = 0.5 * (p[0] + p[2]) + p[1];
    const double r1 = 0.5 * (p[PN] + p[PN + 2]) + p[PN + 1];
    const double r2 = 0.5 * (p[2 * PN] + p[2 * PN + 2]) + p[2 * PN + 1];
    return 0.5 * (r0 + r2) + r1;
  }
}

// NC0: number of finest-level channels (2 only for the adjoint restriction,
// whose second finest channel is the time sum of the cotangent)
#ifndef SG_WPE
#define SG_WPE 1
#endif
template <int D, int TS, int TB, int NT, int STENCIL, int NC0>
__device__ __forceinline__ void restrict_body(const RestrictArgs &A, const double *__restrict__ X,
                                              int lin) {
  using SH = Shape<D, TS, 0>;
  using PD = Pad<D, TS, 0>;
  constexpr int LTS = SH::LTS;
  constexpr int NIN = TS + 2;
  constexpr int INSZ = ipow(NIN, D);
  constexpr int L0 = SH::size(0);
  constexpr int EPT = L0 / NT;                    // fine points per thread
  constexpr int PF = (TB * INSZ + NT - 1) / NT;   // prefetched inputs per thread
  constexpr int NCI = 2 * (LTS + 1);              // in-tile channels, li = 2 r + k
  constexpr int NTAP = NCI * (TB + 1);            // staged tap entries per batch
  constexpr int PT = PD::total;
  static_assert(L0 % NT == 0 && (D == 1 || TS % EPT == 0 || EPT == 1), "tile / block shape");
  static_assert(D == 1 ? EPT == 1 : (NT % TS == 0 && TS % EPT == 0), "column strips");
  static_assert(NTAP <= NT, "one thread per staged tap entry");
  static_assert(SH::upper <= 2 * NT, "two owned upper nodes per thread");
  __shared__ double s_in[TB * INSZ];
  __shared__ double s_lv[TB * PT];
  // taps of the in-tile channels for slabs nb-1 .. nb+TB-1: s_q[li][s] is
  // q0 of slab nb-1+s (-1 outside the chunk), s_w[li][s] the weights of
  // slab nb+s
  __shared__ int s_q[NCI][TB + 1];
  __shared__ double s_w[NCI][TB][3];
  __shared__ int s_qlo[NCI];

  const Geometry g = A.g;
  const int tid = threadIdx.x;
  const int ntileD = (D == 2) ? g.ntile * g.ntile : g.ntile;
  int tile, chunk;
  stream_block(lin, ntileD, g.nchunk, tile, chunk);
  const int tx = tile % g.ntile;
  const int ty = (D == 2) ? tile / g.ntile : 0;
  int n0, n1;
  chunk_span(g, chunk, n0, n1);
  const long long nsp = (D == 2) ? (long long)g.nxf * g.nxf : g.nxf;
  const int R = g.R;
  const bool use_coarse = g.A0 > 1 && A.coarse != nullptr;

  for (int i = tid; i < TB * PT; i += NT) s_lv[i] = 0.0;
  if (tid < NCI) {
    const int r = tid >> 1, k = tid & 1;
    int q = 0;
    if (r <= R) {
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (C.active) q = gld(C.q0, n0);
    }
    s_qlo[tid] = q;
  }

  // fine points of this thread: column strip x, rows y0 .. y0+EPT-1 (2-D)
  const int fx = (D == 2) ? tid % TS : tid;
  const int fy0 = (D == 2) ? (tid / TS) * EPT : 0;
  auto fine_in = [&](int e) {
    return interior(TS * tx + fx, g.nxf) && (D == 1 || interior(TS * ty + fy0 + e, g.nxf));
  };
  // owned upper nodes
  Owned<D, TS, 0> own[2];
  own[0].set(tid);
  own[1].set(tid + NT);
  // tap entry staged by this thread: channel li = tid / (TB+1), slab offset my_s
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
  // input gather of staged element e: slab offset and slab-relative
  // position (-1 outside the interior); recomputed rather than kept in
  // registers
  auto in_slab = [&](int e) {
    const int idx = tid + e * NT;
    return idx < TB * INSZ ? idx / INSZ : TB;
  };
  auto in_pos = [&](int e) {
    const int idx = tid + e * NT;
    const int loc = idx % INSZ;
    const int ix = loc % NIN, iy = loc / NIN;
    const int px = TS * tx - 1 + ix;
    const int py = TS * ty - 1 + iy;
    return (interior(px, g.nxf) && (D == 1 || interior(py, g.nxf)))
               ? (px - 1) + (D == 2 ? (py - 1) * g.nxf : 0)
               : -1;
  };
  double pin[PF];
  int pq = -1;
  double pw0 = 0.0, pw1 = 0.0, pw2 = 0.0;
  // Loads are issued unconditionally from clamped, valid addresses and the
  // unwanted results are discarded with selects: a load inside a divergent
  // branch makes the compiler wait for every earlier load before the next
  // one, which would serialise the prefetch.
  const int *tq0 = my_q0 != nullptr ? my_q0 : A.safe_q0;
  const double *tw = my_q0 != nullptr ? my_w : A.safe_w;
  // (the selects happen when the batch is staged, a loop iteration later)
  auto in_ok = [&](int e, int nb) { return in_slab(e) < min(TB, n1 - nb) && in_pos(e) >= 0; };
  auto tap_ok = [&](int nb) {
    const int n = nb - 1 + my_s;
    return my_q0 != nullptr && n >= n0 && n < n1;
  };
  auto fetch = [&](int nb) {
#pragma unroll
    for (int e = 0; e < PF; ++e)
      pin[e] = X[in_ok(e, nb) ? (long long)(nb + in_slab(e)) * nsp + in_pos(e) : 0];
    const int nc = tap_ok(nb) ? nb - 1 + my_s : 0;
    pq = tq0[nc];
    pw0 = tw[3 * nc];
    pw1 = tw[3 * nc + 1];
    pw2 = tw[3 * nc + 2];
  };

  double racc0[EPT][NC0][3];
  double racc[2][2][3];
#pragma unroll
  for (int e = 0; e < EPT; ++e)
#pragma unroll
    for (int k = 0; k < NC0; ++k) racc0[e][k][0] = racc0[e][k][1] = racc0[e][k][2] = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) racc[i][k][0] = racc[i][k][1] = racc[i][k][2] = 0.0;

  const long long blk = (long long)chunk * ntileD + tile;
  auto part_at = [&](const Channel &C, int li, int r, int q, int j) -> long long {
    return C.part_off + (blk * C.qb + (q - s_qlo[li])) * (long long)SH::size(r) + j;
  };

  fetch(n0);
  __syncthreads();  // zeroed halos and s_qlo
  int last_cnt = 0;
  for (int nb = n0; nb < n1; nb += TB) {
    const int cnt = min(TB, n1 - nb);
    last_cnt = cnt;
    // (1) staged batch -> LDS, then start fetching the next batch
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int idx = tid + e * NT;
      if (idx < TB * INSZ) s_in[idx] = in_ok(e, nb) ? pin[e] : 0.0;
    }
    if (tid < NTAP) {
      const int li = tid / (TB + 1);
      const bool ok = tap_ok(nb);
      s_q[li][my_s] = ok ? pq : -1;
      if (my_s > 0) {
        s_w[li][my_s - 1][0] = ok ? pw0 : 0.0;
        s_w[li][my_s - 1][1] = ok ? pw1 : 0.0;
        s_w[li][my_s - 1][2] = ok ? pw2 : 0.0;
      }
    }
    __syncthreads();
    if (nb + TB < n1) fetch(nb + TB);
    // (2) fine level: optional mass stencil, accumulation, level-0 array
    for (int s = 0; s < cnt; ++s) {
      const double *in = s_in + s * INSZ;
      double m[EPT];
      if (D == 1) {
        m[0] = STENCIL ? (fine_in(0) ? A.sx * (in[fx] + in[fx + 2] + 4.0 * in[fx + 1]) : 0.0)
                       : in[fx + 1];
      } else if (STENCIL) {
        double h[EPT + 2];
#pragma unroll
        for (int i = 0; i < EPT + 2; ++i) {
          const double *row = in + (fy0 + i) * NIN + fx;
          h[i] = row[0] + row[2] + 4.0 * row[1];
        }
        const double sxy = A.sx * A.sy;
#pragma unroll
        for (int e = 0; e < EPT; ++e)
          m[e] = fine_in(e) ? sxy * (h[e] + h[e + 2] + 4.0 * h[e + 1]) : 0.0;
      } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) m[e] = in[(fy0 + e + 1) * NIN + fx + 1];
      }
      double *l0 = s_lv + s * PT;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        if (D == 1) l0[fx + 1] = m[0];
        else l0[(fy0 + e + 1) * PD::pn(0) + fx + 1] = m[e];
      }
#pragma unroll
      for (int k = 0; k < NC0; ++k) {
        if (!A.ch[(g.J - 1) * 2 + k].active) continue;
        const double w0 = s_w[k][s][0], w1 = s_w[k][s][1], w2 = s_w[k][s][2];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          racc0[e][k][0] += w0 * m[e];
          racc0[e][k][1] += w1 * m[e];
          racc0[e][k][2] += w2 * m[e];
        }
      }
    }
    __syncthreads();
    // (3) levels r = 1..R: owners restrict from level r-1 and accumulate
#pragma unroll
    for (int r = 1; r <= LTS; ++r) {
      if (r > R) break;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (own[i].r != r) continue;
        for (int s = 0; s < cnt; ++s) {
          const double *src = s_lv + s * PT + PD::poff(r - 1);
          const double v = full_weight<D>(src, PD::pn(r - 1), own[i].jx, own[i].jy);
          s_lv[s * PT + PD::poff(r) + (D == 2 ? (own[i].jy + 1) * PD::pn(r) : 0) + own[i].jx + 1] = v;
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int li = 2 * r + k;
            const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
            if (!C.active) continue;
            const int q0n = s_q[li][s + 1], qp = s_q[li][s];
            if (qp >= 0 && q0n > qp) {
              A.part[part_at(C, li, r, qp, own[i].j)] = racc[i][k][0];
              racc[i][k][0] = racc[i][k][1];
              racc[i][k][1] = racc[i][k][2];
              racc[i][k][2] = 0.0;
            }
            racc[i][k][0] += s_w[li][s][0] * v;
            racc[i][k][1] += s_w[li][s][1] * v;
            racc[i][k][2] += s_w[li][s][2] * v;
          }
          if (r == R && use_coarse)
            A.coarse[((long long)tile * g.ntf + nb + s) * SH::size(r) + own[i].j] = v;
        }
      }
      __syncthreads();
    }
  }
  // final flush of the open time nodes (s_q still holds the last batch; the
  // level-J channels keep one window per time chunk, so their nodes are the
  // chunk's q0 + 0, 1, 2, stored relative to it)
#pragma unroll
  for (int k = 0; k < NC0; ++k) {
    const Channel &C = A.ch[(g.J - 1) * 2 + k];
    if (!C.active) continue;
#pragma unroll
    for (int o = 0; o < 3; ++o)
#pragma unroll
      for (int e = 0; e < EPT; ++e)
        A.part[part_at(C, k, 0, s_qlo[k] + o, (D == 2 ? (fy0 + e) * TS : 0) + fx)] =
            racc0[e][k][o];
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = own[i].r;
    if (r == 0 || r > R) continue;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int li = 2 * r + k;
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (!C.active) continue;
      const int ql = s_q[li][last_cnt];
#pragma unroll
      for (int o = 0; o < 3; ++o)
        if (ql + o < C.nq) A.part[part_at(C, li, r, ql + o, own[i].j)] = racc[i][k][o];
    }
  }
}

template <int D, int TS, int TB, int NT, int STENCIL, int NC0>
__global__ void __launch_bounds__(NT, SG_WPE) k_restrict(const RestrictArgs A) {
  restrict_body<D, TS, TB, NT, STENCIL, NC0>(A, A.X, block_lin());
}

// Read-only tables (tap offsets and weights) through the scalar cache: a load
// from the constant address space with a wave-uniform address becomes a
// scalar load into SGPRs.  The tables are never written by these kernels.
typedef const __attribute__((address_space(4))) int cint_t;
typedef const __attribute__((address_space(4))) TapEntry ctap_t;
__device__ __forceinline__ int ld_const(const int *p, int i) { return ((cint_t *)p)[i]; }
__device__ __forceinline__ TapEntry ld_const(const TapEntry *p, long long i) {
  ctap_t *q = (ctap_t *)p + i;
  TapEntry t;
  t.w[0] = q->w[0];
  t.w[1] = q->w[1];
  t.w[2] = q->w[2];
  t.base = q->base;
  return t;
}

// Order the LDS accesses of one wave around this point (the lanes of a wave
// see each other's LDS stores in program order; this stops the compiler from
// moving accesses across it).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-slab tap block of the 16 x 16 streaming kernels: NCI entries of four
// doubles (three weights, then the entry's base), copied into the wave's LDS
// at the top of every slab.  Lane l < 4 NCI prefetches double l of the next
// slab's block one slab ahead, so the weights never wait on memory; every
// lane then reads the taps of its own level.  Entry 0 carries in its base the
// bit mask of the entries whose window moves on at this slab.
template <int NCI>
struct SlabTaps {
  static_assert(4 * NCI <= 64, "one tap double per lane");
  const double *tab;
  double next;
  __device__ void fetch(const TapEntry *taps, int n, int lane) {
    tab = reinterpret_cast<const double *>(taps);
    next = tab[(long long)n * (4 * NCI) + min(lane, 4 * NCI - 1)];
  }
  __device__ void stage(double *s_t, int lane) const {
    if (lane < 4 * NCI) s_t[lane] = next;
  }
};
// A per-lane offset the compiler must treat as new in every iteration, so
// that it adds it to a uniform row pointer where the load happens instead of
// keeping a hoisted 64-bit address per lane live across the slab loop.
__device__ __forceinline__ int lane_off(int o) {
  asm volatile("" : "+v"(o));
  return o;
}

// Materialise a loaded value at this point of the program (the empty asm is
// ordered with the stores around it, so the wait for the load lands here).
__device__ __forceinline__ void take(double &v) { asm volatile("" : "+v"(v)); }

// moving-window mask of the staged slab (uniform)
__device__ __forceinline__ int slab_moves(const double *s_t) {
  return __builtin_amdgcn_readfirstlane((int)__double_as_longlong(s_t[3]));
}

// Upper levels r = 1..4 of a 16 x 16 tile in the per-wave restriction: level
// r keeps its nodes(r)^2 values at (jy + 1) pitch(r) + jx + 1 with zero halo
// entries, as Pad does, but with even pitches, so that the first two entries
// of every full-weighting row are one aligned 16-byte read.
__host__ __device__ constexpr int up16_nodes(int r) { return (16 >> r) + 1; }
__host__ __device__ constexpr int up16_pitch(int r) { return (up16_nodes(r) + 3) & ~1; }
__host__ __device__ constexpr int up16_off(int r) {
  return r <= 1 ? 0 : up16_off(r - 1) + up16_pitch(r - 1) * up16_pitch(r - 1);
}
struct Up16 {
  __host__ __device__ static constexpr int nodes(int r) { return up16_nodes(r); }
  __host__ __device__ static constexpr int pitch(int r) { return up16_pitch(r); }
  __host__ __device__ static constexpr int off(int r) { return up16_off(r); }
  static constexpr int total = up16_off(5);
};
static_assert(Up16::pitch(1) >= 2 * Up16::nodes(2) + 1 && Up16::pitch(2) >= 2 * Up16::nodes(3) + 1 &&
                  Up16::pitch(3) >= 2 * Up16::nodes(4) + 1,
              "full-weighting windows inside the padded level below");

// Full weighting from a padded level with an even pitch P; p = the window's
// corner (even offset).  Same arithmetic as full_weight<2>.
__device__ __forceinline__ double full_weight_pairs(const double *p, int P) {
  double r[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double2 a = *reinterpret_cast<const double2 *>(p + i * P);
    r[i] = 0.5 * (a.x + p[i * P + 2]) + a.y;
  }
  return 0.5 * (r[0] + r[2]) + r[1];
}

// Value of lane l - 1 within each row of 16 lanes (DPP row_shr:1; lanes 0 and
// 16, 32, 48 read zero).
__device__ __forceinline__ double row_shr1(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x111, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x111, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Value of lane `src` (mod 64) through the LDS crossbar (no LDS memory).
__device__ __forceinline__ double lane_value(double v, int src) {
  const int a = src << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Upper nodes of a wave's 16 x 16 tile in the per-wave restriction.  Slot 0
// of lane (lx, ly) = (l % 8, l / 8) is the level-1 node (lx, ly), which the
// lane builds in registers from its own 2 x 2 fine block and those of its
// left and upper neighbours.  Slot 1 of lane u: the level-1 nodes (8, u) for
// u < 9 and (u - 9, 8) for 9 <= u < 17, then the nodes of levels 2, 3, 4 in
// row-major order (lanes 17 .. 54), none above.  j is the row-major index in
// the level, as in the partial-block layout.
struct Slot16 {
  int r = 0, j = 0, jx = 0, jy = 0;
  __device__ void set0(int lane) {
    r = 1;
    jx = lane & 7;
    jy = lane >> 3;
    j = jy * Up16::nodes(1) + jx;
  }
  __device__ void set1(int u) {
    r = 0;
    if (u < 9) {
      r = 1, jx = 8, jy = u;
    } else if (u < 17) {
      r = 1, jx = u - 9, jy = 8;
    } else {
      int v = u - 17;
#pragma unroll
      for (int rr = 2; rr <= 4; ++rr) {
        const int n = Up16::nodes(rr);
        if (r == 0 && v < n * n) {
          r = rr, jx = v % n, jy = v / n;
        } else if (r == 0) {
          v -= n * n;
        }
      }
    }
    j = r ? jy * Up16::nodes(r) + jx : 0;
  }
};

// 2-D restriction with one 16 x 16 tile per wave.  Every wave streams the
// slabs of its own tile, so the slab loop has no workgroup barrier; the four
// waves of a workgroup take a 2 x 2 block of tiles, which share halo rows in
// the caches.  Lane l owns the 2 x 2 block of fine nodes at (2 (l % 8),
// 2 (l / 8)).  Per slab it forms the fine values (through the mass stencil
// from an LDS copy of the 18 x 18 input window, or straight from memory),
// then its shares of the four level-1 nodes around the block: the shares
// from the left neighbour arrive by a DPP row shift, those from the row of
// blocks above through the LDS crossbar, so level 1 is complete in
// registers.  Level 1 goes to LDS once; levels 2..4 follow by full weighting
// there.  Same outputs and partial-block layout as k_restrict<2, 16, ...>.
// Three workgroups per CU.
#ifndef SG_WPEW
#define SG_WPEW 3
#endif
template <int STENCIL, int NC0>
__device__ __forceinline__ void restrict_w_body(const RestrictArgs &A, const double *__restrict__ X,
                                                int lin) {
  constexpr int TS = 16, LTS = 4, NIN = TS + 2, INSZ = NIN * NIN, NP = 24;
  // loads in flight per lane: the input window (mass stencil) or the block
  constexpr int PF = STENCIL ? (INSZ + 63) / 64 : 4;
  using SH = Shape<2, TS, 0>;
  static_assert(INSZ % 2 == 0, "16-byte aligned rows of the staged input");
  __shared__ __align__(16) double s_in_w[4][STENCIL ? NIN * NP : 2];
  __shared__ __align__(16) double s_lv_w[4][Up16::total];
  constexpr int NCI = 2 * (LTS + 1);  // in-tile channels li = 2 r + k
  __shared__ __align__(16) double s_t_w[4][4 * NCI];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *s_in = s_in_w[wave];
  double *s_lv = s_lv_w[wave];
  double *s_t = s_t_w[wave];

  const Geometry g = A.g;
  const int nt = g.ntile, ng = (nt + 1) >> 1;
  int grp, chunk;
  stream_block(lin, ng * ng, g.nchunk, grp, chunk);
  const int tx = 2 * (grp % ng) + (wave & 1), ty = 2 * (grp / ng) + (wave >> 1);
  if (tx >= nt || ty >= nt) return;  // no workgroup barrier below
  const int tile = ty * nt + tx, ntileD = nt * nt;
  int n0, n1;
  chunk_span(g, chunk, n0, n1);
  const long long nsp = (long long)g.nxf * g.nxf;
  const int R = g.R;
  const bool use_coarse = g.A0 > 1 && A.coarse != nullptr;
  const long long blk = (long long)chunk * ntileD + tile;

  for (int i = lane; i < Up16::total; i += 64) s_lv[i] = 0.0;

  // fine nodes (fx, fy) = (2 lx + c, 2 ly + b) of this lane
  const int lx = lane & 7, ly = lane >> 3;
  bool fin[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      fin[b][c] = interior(TS * tx + 2 * lx + c, g.nxf) && interior(TS * ty + 2 * ly + b, g.nxf);
  Slot16 own[2];
  own[0].set0(lane);
  own[1].set1(lane);

  // load e of this lane: slab-relative offset, -1 outside the interior
  int pos[PF];
#pragma unroll
  for (int e = 0; e < PF; ++e) {
    if (STENCIL) {
      const int idx = lane + 64 * e;
      const int ix = idx % NIN, iy = idx / NIN;
      const int px = TS * tx - 1 + ix, py = TS * ty - 1 + iy;
      pos[e] = (idx < INSZ && interior(px, g.nxf) && interior(py, g.nxf))
                   ? (py - 1) * g.nxf + (px - 1) : -1;
    } else {
      const int b = e >> 1, c = e & 1;
      pos[e] = fin[b][c] ? (TS * ty + 2 * ly + b - 1) * g.nxf + (TS * tx + 2 * lx + c - 1) : -1;
    }
  }
  double pin[PF];
  double cur[2][2];  // the lane's block of the current slab (identity stencil)
  // unconditional loads from valid addresses; unwanted values are replaced
  // by zeros when staged (a load in a divergent branch would serialise them)
  auto fetch = [&](int n) {
#pragma unroll
    for (int e = 0; e < PF; ++e) pin[e] = X[pos[e] >= 0 ? (long long)n * nsp + pos[e] : 0];
  };

  // fine-level accumulators; a second finest channel (the adjoint's time sum
  // of the cotangent) has weights (w, 0, 0) and keeps one node
  double racc0[2][2][3];
  double rsum[2][2];
  double racc[2][2][3];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      racc0[b][c][0] = racc0[b][c][1] = racc0[b][c][2] = 0.0;
      rsum[b][c] = 0.0;
    }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) racc[i][k][0] = racc[i][k][1] = racc[i][k][2] = 0.0;

  // partial-block entry of row `base` (channel offset + chunk-relative row)
  auto part_at = [&](const Channel &C, long long base, int r, int j) -> long long {
    return base + blk * C.qb * (long long)SH::size(r) + j;
  };

  // tap entry of slot i: entries 2 r, 2 r + 1 of its level (0 when idle)
  int tslot[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) tslot[i] = (own[i].r >= 1 && own[i].r <= R) ? 8 * own[i].r : 0;
  // slot 1: the corner of its full-weighting window in the level below, that
  // level's pitch, and its own entry (levels >= 2); a level-1 node only reads
  // its entry
  int fw1 = 0, pw1 = 0, st1 = 0;
  if (own[1].r >= 1) {
    st1 = Up16::off(own[1].r) + (own[1].jy + 1) * Up16::pitch(own[1].r) + own[1].jx + 1;
    if (own[1].r >= 2) {
      pw1 = Up16::pitch(own[1].r - 1);
      fw1 = Up16::off(own[1].r - 1) + 2 * own[1].jy * pw1 + 2 * own[1].jx;
    }
  }
  SlabTaps<NCI> tp;
  tp.fetch(A.taps, n0, lane);

  // the input and taps of slab n + 1 are staged at the end of slab n, before
  // its stores: loads and stores share one completion counter, so a store
  // issued just before a wait for loads would hold that wait up
  auto stage_next = [&]() {
    if (STENCIL) {
#pragma unroll
      for (int e = 0; e < PF; ++e) {
        const int idx = lane + 64 * e;
        if (idx < INSZ) s_in[(idx / NIN) * NP + idx % NIN] = pos[e] >= 0 ? pin[e] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < PF; ++e) {
        cur[e >> 1][e & 1] = pos[e] >= 0 ? pin[e] : 0.0;
        take(cur[e >> 1][e & 1]);
      }
    }
    tp.stage(s_t, lane);
  };
  fetch(n0);
  stage_next();
  for (int n = n0; n < n1; ++n) {
    if (n + 1 < n1) {
      fetch(n + 1);
      tp.fetch(A.taps, n + 1, lane);
    }
    wave_sync();
    // (1) fine level: the mass stencil over the 4 x 4 input window of the
    // lane's 2 x 2 block, one row at a time (rows i = 0..3 are input rows
    // 2 ly + i), or the block itself
    double m[2][2];
    if (STENCIL) {
      // row sums h_c(i) = v(i, c) + v(i, c + 2) + 4 v(i, c + 1), folded into
      // the two output rows as they arrive
      double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double2 *p = reinterpret_cast<const double2 *>(s_in + (2 * ly + i) * NP + 2 * lx);
        const double2 a0 = p[0], a1 = p[1];
        const double h0 = a0.x + a1.x + 4.0 * a0.y, h1 = a0.y + a1.y + 4.0 * a1.x;
        // output row b takes input rows b, b+1, b+2 with weights 1, 4, 1
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int d = i - b;
          if (d < 0 || d > 2) continue;
          const double wt = d == 1 ? 4.0 : 1.0;
          acc[b][0] += wt * h0;
          acc[b][1] += wt * h1;
        }
      }
      const double sxy = A.sx * A.sy;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) m[b][c] = fin[b][c] ? sxy * acc[b][c] : 0.0;
    } else {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) m[b][c] = cur[b][c];
    }
    const TapEntry *tn = A.taps + (long long)n * NCI;
    {  // level-J channel (zero weights when inactive)
      const double2 w01 = *reinterpret_cast<const double2 *>(s_t);
      const double w2 = s_t[2];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          racc0[b][c][0] += w01.x * m[b][c];
          racc0[b][c][1] += w01.y * m[b][c];
          racc0[b][c][2] += w2 * m[b][c];
        }
    }
    if (NC0 == 2) {
      const double w = s_t[4];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) rsum[b][c] += w * m[b][c];
    }
    // (2) level 1 in registers.  The block's shares: A to node (lx, ly), Ex
    // to (lx + 1, ly), Ey to (lx, ly + 1), Exy to (lx + 1, ly + 1) (full
    // weighting: 1 at the node, 1/2 on its edges, 1/4 on its corners).  X1
    // and Y1 collect what the lane's row of blocks gives to nodes (lx, ly) and
    // (lx, ly + 1), adding the left neighbour's shares; lanes lx = 7 also hold
    // the row's shares of the column-8 nodes (Ex, Exy).
    double val[2] = {0.0, 0.0};
    if (R >= 1) {
      const double exy = 0.25 * m[1][1];
      const double a1 = m[0][0] + 0.5 * (m[0][1] + m[1][0]) + exy;
      const double ex = 0.5 * m[0][1] + exy, ey = 0.5 * m[1][0] + exy;
      const double exl = row_shr1(ex), exyl = row_shr1(exy);  // all lanes take part
      const double x1 = lx ? a1 + exl : a1;
      const double y1 = lx ? ey + exyl : ey;
      const double up = lane_value(y1, lane - 8), upe = lane_value(exy, lane - 8);
      const double l1 = ly ? x1 + up : x1;     // node (lx, ly)
      const double l1e = ly ? ex + upe : ex;   // node (8, ly) in lanes lx = 7
      val[0] = l1;
      double *v1 = s_lv + Up16::off(1);
      constexpr int P1 = Up16::pitch(1);
      v1[(ly + 1) * P1 + lx + 1] = l1;
      // column 8 from lanes lx = 7, row 8 from lanes ly = 7 (lx < 7): only
      // the row's own shares reach these nodes
      if (lx == 7 || ly == 7)
        v1[lx == 7 ? (ly + 1) * P1 + 9 : 9 * P1 + lx + 1] = lx == 7 ? l1e : y1;
      if (lane == 63)  // nodes (7, 8) and (8, 8): adjacent, 16-byte aligned
        *reinterpret_cast<double2 *>(v1 + 9 * P1 + 8) = make_double2(y1, exy);
      static_assert((9 * Up16::pitch(1) + 8) % 2 == 0, "aligned pair");
    }
    // (3) levels 2..R by full weighting in LDS (slot 1 owners); slot-1
    // level-1 nodes read their value
    if (R >= 1) {
      wave_sync();
      if (own[1].r == 1) val[1] = s_lv[lane_off(st1)];
#pragma unroll
      for (int r = 2; r <= LTS; ++r) {
        if (r > R) break;
        if (r > 2) wave_sync();
        if (own[1].r == r) {
          val[1] = full_weight_pairs(s_lv + lane_off(fw1), pw1);
          s_lv[lane_off(st1)] = val[1];
        }
      }
    }
    // windows that close their oldest time node at this slab
    const int mv = slab_moves(s_t);
    if (mv != 0) {
#pragma unroll
      for (int r = 1; r <= LTS; ++r) {
        if (r > R) break;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          if (!((mv >> (2 * r + k)) & 1)) continue;
          const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
          const long long base = ld_const(tn, 2 * r + k).base;
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            if (own[i].r != r) continue;
            A.part[part_at(C, base, r, own[i].j)] = racc[i][k][0];
            racc[i][k][0] = racc[i][k][1];
            racc[i][k][1] = racc[i][k][2];
            racc[i][k][2] = 0.0;
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double *t = s_t + tslot[i];
      const double2 a0 = *reinterpret_cast<const double2 *>(t);
      const double2 a1 = *reinterpret_cast<const double2 *>(t + 2);
      const double2 b0 = *reinterpret_cast<const double2 *>(t + 4);
      const double2 b1 = *reinterpret_cast<const double2 *>(t + 6);
      racc[i][0][0] += a0.x * val[i];
      racc[i][0][1] += a0.y * val[i];
      racc[i][0][2] += a1.x * val[i];
      racc[i][1][0] += b0.x * val[i];
      racc[i][1][1] += b0.y * val[i];
      racc[i][1][2] += b1.x * val[i];
    }
    if (n + 1 < n1) stage_next();
    wave_sync();
    if (use_coarse) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
        if (own[i].r == R)
          (A.coarse + ((long long)tile * g.ntf + n) * SH::size(R))[lane_off(own[i].j)] = val[i];
    }
  }
  // final flush of the open time nodes (level-J channels: one window per
  // time chunk, stored relative to its q0)
#pragma unroll
  for (int k = 0; k < NC0; ++k) {
    const Channel &C = A.ch[(g.J - 1) * 2 + k];
    if (!C.active) continue;
#pragma unroll
    for (int o = 0; o < 3; ++o)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          A.part[part_at(C, C.part_off + (long long)o * SH::size(0), 0,
                         (2 * ly + b) * TS + 2 * lx + c)] =
              k == 0 ? racc0[b][c][o] : (o == 0 ? rsum[b][c] : 0.0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = own[i].r;
    if (r == 0 || r > R) continue;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (!C.active) continue;
      const int qlo = ld_const(C.q0, n0), ql = ld_const(C.q0, n1 - 1);
#pragma unroll
      for (int o = 0; o < 3; ++o)
        if (ql + o < C.nq)
          A.part[part_at(C, C.part_off + (long long)(ql + o - qlo) * SH::size(r), r, own[i].j)] =
              racc[i][k][o];
    }
  }
}

template <int STENCIL, int NC0>
__global__ void __launch_bounds__(256, SG_WPEW) k_restrict_w(const RestrictArgs A) {
  restrict_w_body<STENCIL, NC0>(A, A.X, block_lin());
}

// Index of the last of n items (ascending .start) whose start is <= gid.
// A binary search on the wave's first thread (wave-uniform: scalar loads,
// whose upper levels every wave shares in the scalar cache) finds the item
// there; a lane then steps on only across the rare item boundaries inside
// its wave.  Batches of many problems hold thousands of items, so a scan
// over the starts would cost each wave far more than its own work.
template <class T>
__device__ __forceinline__ int find_item(const T *items, int n, long long gid, long long gw) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].start <= gw) lo = mid; else hi = mid - 1;
  }
  int it = lo;
  while (it + 1 < n && items[it + 1].start <= gid) ++it;
  return it;
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
__device__ __forceinline__ void reduce_body(const Geometry &g, const Channel *__restrict__ ch,
                                            const double *__restrict__ part,
                                            const WorkItem *__restrict__ items, int nitems,
                                            long long total, long long gid, long long gw) {
  using SH = Shape<D, TS, 0>;
  const int it = find_item(items, nitems, gid, gw);
  if (gid >= total) return;
  const Channel &C = ch[items[it].ch];
  // the channel's fields once, ahead of the loops (a field read inside a
  // conditional loop body is read again on every trip, each read one more
  // memory round trip before the partial it addresses)
  const int a = C.a, qb = C.qb;
  const long long part_off = C.part_off;
  const int *const q0 = C.q0;
  double *const data = C.data;
  const double scale = C.scale;
  const long long loc = gid - items[it].start;
  const int r = g.J - a;
  const int na = (1 << a) - 1;
  // 32-bit index arithmetic: a channel holds fewer than 2^31 coefficients
  const int nsp = (D == 2) ? na * na : na;
  const int q = (int)loc / nsp;
  const int K = (int)loc - q * nsp;
  const int Py = (D == 2) ? K / na + 1 : 0;
  const int Px = (D == 2) ? K - (Py - 1) * na + 1 : K + 1;
  const int nr = SH::nodes(r), sz = SH::size(r);
  const int ntileD = (D == 2) ? g.ntile * g.ntile : g.ntile;
  int tx0, tx1, ty0 = 0, ty1 = 0;
  tile_range(TS, r, Px, g.ntile, tx0, tx1);
  if (D == 2) tile_range(TS, r, Py, g.ntile, ty0, ty1);
  // the node's (up to 2 x 2) tiles: offsets within a partial block, or -1
  constexpr int NY = (D == 2) ? 2 : 1;
  long long toff[NY][2];
#pragma unroll
  for (int dy = 0; dy < NY; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const int ty = ty0 + dy, tx = tx0 + dx;
      const int jy = (D == 2) ? Py - tile_lo(TS, ty, r, 0) : 0;
      const int jx = Px - tile_lo(TS, tx, r, 0);
      const bool ok = ty <= ty1 && tx <= tx1 && jy >= 0 && jy < nr && jx >= 0 && jx < nr;
      toff[dy][dx] = ok ? (long long)(ty * g.ntile + tx) * qb * sz + jy * nr + jx : -1;
    }
  // per chunk whose window holds q: its partials of those tiles, loaded
  // together and added in the fixed order ty, tx
  double acc = 0.0;
  for (int c = 0; c < g.nchunk; ++c) {
    int cn0, cn1;
    chunk_span(g, c, cn0, cn1);
    const int qlo = gld(q0, cn0), qhi = gld(q0, cn1 - 1) + 2;
    if (q < qlo || q > qhi) continue;
    const long long base = part_off + ((long long)c * ntileD * qb + (q - qlo)) * (long long)sz;
    double v[NY][2];
#pragma unroll
    for (int dy = 0; dy < NY; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const long long o = toff[dy][dx];
        const double x = part[o >= 0 ? base + o : base];
        v[dy][dx] = o >= 0 ? x : 0.0;
      }
#pragma unroll
    for (int dy = 0; dy < NY; ++dy) {
      acc += v[dy][0];
      acc += v[dy][1];
    }
  }
  gst(data, loc, scale * acc);
}

template <int D, int TS>
__global__ void k_reduce(const Geometry g, const Channel *__restrict__ ch,
                         const double *__restrict__ part,
                         const WorkItem *__restrict__ items, int nitems,
                         long long total) {
  reduce_body<D, TS>(g, ch, part, items, nitems, total, gid64(),
                     wave_gid0((long long)blockIdx.x * blockDim.x));
}

// first index n with q0[n] >= v (q0 nondecreasing)
__device__ __forceinline__ int lower_bound_q(const int *q0, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (gld(q0, mid) < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Offset of level a inside a slab's coarse-level block (levels 1 .. A0-1).
__host__ __device__ inline long long coarse_off(int d, int a) {
  long long o = 0;
  for (int l = 1; l < a; ++l) {
    const long long n = (1 << l) - 1;
    o += d == 2 ? n * n : n;
  }
  return o;
}

// One block per slab: the level-A0 values of slab n from the per-slab tile
// partials of the restriction (a level-A0 node is shared by the tiles t = P-1
// and t = P per axis, whose top in-tile level has two nodes per axis), then
// full weighting down to level 1.
template <int D>
__device__ __forceinline__ void coarse_pyramid_body(const Geometry &g,
                                                    const double *__restrict__ cp,
                                                    double *__restrict__ SL, int n) {
  constexpr int MAXN = kCoarseMax;  // doubles per ping-pong level (checked by the plan)
  __shared__ double s_a[MAXN], s_b[MAXN];
  const int A0 = g.A0;
  const int n0a = (1 << A0) - 1;
  const int nsp0 = (D == 2) ? n0a * n0a : n0a;
  const long long tot = coarse_off(D, A0);
  constexpr int SZ = (D == 2) ? 4 : 2;  // top in-tile level of a tile
  for (int K = threadIdx.x; K < nsp0; K += blockDim.x) {
    const int Py = (D == 2) ? K / n0a + 1 : 0;
    const int Px = (D == 2) ? K - (Py - 1) * n0a + 1 : K + 1;
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
    s_a[K] = acc;
  }
  __syncthreads();
  double *cur = s_a, *nxt = s_b;
  for (int a = A0 - 1; a >= 1; --a) {
    const int na = (1 << a) - 1, nf = (1 << (a + 1)) - 1;
    const int nspa = (D == 2) ? na * na : na;
    for (int i = threadIdx.x; i < nspa; i += blockDim.x) {
      const int Kx = i % na + 1, Ky = (D == 2) ? i / na + 1 : 0;  // level-a node
      double v = 0.0;
      for (int dy = (D == 2 ? -1 : 0); dy <= (D == 2 ? 1 : 0); ++dy) {
        const double wy = dy == 0 ? 1.0 : 0.5;
        const int fy = 2 * Ky + dy;  // level a+1 node, interior 1..nf
        double row = 0.0;
        for (int dx = -1; dx <= 1; ++dx) {
          const int fx = 2 * Kx + dx;
          row += (dx == 0 ? 1.0 : 0.5) * cur[(D == 2 ? (fy - 1) * nf : 0) + fx - 1];
        }
        v += wy * row;
      }
      nxt[i] = v;
      SL[(long long)n * tot + coarse_off(D, a) + i] = v;
    }
    __syncthreads();
    double *t = cur; cur = nxt; nxt = t;
  }
}

template <int D>
__global__ void __launch_bounds__(256) k_coarse_pyramid(const Geometry g,
                                                        const double *__restrict__ cp,
                                                        double *__restrict__ SL) {
  coarse_pyramid_body<D>(g, cp, SL, blockIdx.x);
}

// Channels of the levels a < A0: sum over the slabs that touch time node q
// of the tap weight times the slab's level-a restriction.
template <int D>
__device__ __forceinline__ void coarse_restrict_body(const Geometry &g,
                                                     const Channel *__restrict__ ch,
                                                     const double *__restrict__ SL,
                                                     const WorkItem *__restrict__ items,
                                                     int nitems, long long total, long long gid,
                                                     long long gw) {
  const int it = find_item(items, nitems, gid, gw);
  if (gid >= total) return;
  const Channel &C = ch[items[it].ch];
  const int a = C.a;  // the channel's fields once, ahead of the loop
  const int *const q0 = C.q0;
  const double *const w = C.w;
  double *const data = C.data;
  const double scale = C.scale;
  const long long loc = gid - items[it].start;
  const int na = (1 << a) - 1;
  const int nsp = (D == 2) ? na * na : na;
  const int q = (int)loc / nsp;  // coarse channels hold fewer than 2^31 values
  const int K = (int)loc - q * nsp;
  const long long tot = coarse_off(D, g.A0), off = coarse_off(D, a) + K;
  const int nlo = lower_bound_q(q0, g.ntf, q - 2);
  const int nhi = lower_bound_q(q0, g.ntf, q + 1);  // exclusive
  // q0 is nondecreasing, so every slab in [nlo, nhi) has q - 2 <= q0[n] <= q:
  // no test in the loop, whose loads can then be in flight together
  double acc = 0.0;
#pragma unroll 4
  for (int n = nlo; n < nhi; ++n)
    acc += gld(w, 3 * n + (q - gld(q0, n))) * SL[(long long)n * tot + off];
  gst(data, loc, scale * acc);
}

template <int D>
__global__ void k_coarse_restrict(const Geometry g, const Channel *__restrict__ ch,
                                  const double *__restrict__ SL,
                                  const WorkItem *__restrict__ items, int nitems,
                                  long long total) {
  coarse_restrict_body<D>(g, ch, SL, items, nitems, total, gid64(),
                          wave_gid0((long long)blockIdx.x * blockDim.x));
}

// ---------------------------------------------------------- prolongation ---

// C[n][K0] at the interior level-A0 nodes: sum over the channels of levels
// a < A0 of their time-evaluated values, interpolated linearly.  One block
// per slab builds the nodal values level by level, coarse to fine (the P1
// interpolation from level a to level A0 is the composition of the
// interpolations between consecutive levels): level a takes its channels'
// values at slab n plus the interpolation of level a-1; level A0 only the
// interpolation.
template <int D>
__device__ __forceinline__ void prolong_coarse_body(const Geometry &g,
                                                    const Channel *__restrict__ ch,
                                                    double *__restrict__ Cout, int n) {
  // level A0-1 has fewer than a quarter (a half in 1-D) of the level-A0
  // nodes, which the plan keeps within kCoarseMax
  constexpr int MAXN = kCoarseMax / (D == 2 ? 4 : 2);
  __shared__ double s_a[MAXN], s_b[MAXN];
  const int A0 = g.A0;
  double *cur = s_a, *nxt = s_b;
  for (int a = 1; a <= A0; ++a) {
    const int na = (1 << a) - 1, nc = (1 << (a - 1)) - 1;
    const int nspa = (D == 2) ? na * na : na;
    // value of level a-1 at its node (X, Y); zero on the boundary
    auto at = [&](int X, int Y) -> double {
      if (X < 1 || X > nc || (D == 2 && (Y < 1 || Y > nc))) return 0.0;
      return cur[(D == 2 ? (Y - 1) * nc : 0) + X - 1];
    };
    // the level's two channels, read once per level (uniform)
    const Channel &C0 = ch[(a - 1) * 2], &C1 = ch[(a - 1) * 2 + 1];
    const bool act[2] = {a < A0 && C0.active != 0, a < A0 && C1.active != 0};
    const int *const cq0[2] = {C0.q0, C1.q0};
    const double *const cw[2] = {C0.w, C1.w};
    const double *const cdata[2] = {C0.data, C1.data};
    const double cscale[2] = {C0.scale, C1.scale};
    for (int i = threadIdx.x; i < nspa; i += blockDim.x) {
      const int Px = i % na + 1, Py = (D == 2) ? i / na + 1 : 0;
      double v = 0.0;
      if (a > 1) {
        const int xl = Px >> 1, xh = (Px + 1) >> 1;  // equal at even nodes
        if (D == 2) {
          const int yl = Py >> 1, yh = (Py + 1) >> 1;
          v = 0.25 * (at(xl, yl) + at(xh, yl) + at(xl, yh) + at(xh, yh));
        } else {
          v = 0.5 * (at(xl, 0) + at(xh, 0));
        }
      }
      if (a == A0) {
        Cout[(long long)n * nspa + i] = v;
        continue;
      }
      for (int k = 0; k < 2; ++k) {
        if (!act[k]) continue;
        const int q0n = gld(cq0[k], n);
        double sv = 0.0;
        for (int kk = 0; kk < 3; ++kk) {
          const double w = gld(cw[k], 3 * n + kk);
          if (w == 0.0) continue;  // (a window past the last time node)
          sv += w * gld(cdata[k], (long long)(q0n + kk) * nspa + i);
        }
        v += cscale[k] * sv;
      }
      nxt[i] = v;
    }
    __syncthreads();
    double *t = cur;
    cur = nxt;
    nxt = t;
  }
}

template <int D>
__global__ void __launch_bounds__(256) k_prolong_coarse(const Geometry g,
                                                        const Channel *__restrict__ ch,
                                                        double *__restrict__ Cout) {
  prolong_coarse_body<D>(g, ch, Cout, blockIdx.x);
}

// NC0: number of finest-level channels (2 only for the u0/v0 field pass)
template <int D, int TS, int TB, int NT, int MODE, int NC0>
__device__ __forceinline__ void prolong_body(const ProlongArgs &A, const double *__restrict__ base,
                                             double *__restrict__ out, int lin) {
  using SH = Shape<D, TS, MODE>;
  constexpr int LTS = SH::LTS;
  constexpr int L0 = SH::size(0);
  constexpr int EPT0 = (L0 + NT - 1) / NT;
  constexpr int UP = SH::upper;
  constexpr int NO = ipow(TS, D);          // output points per slab
  constexpr int EPTO = NO / NT;
  constexpr int NF = TS + 2 * MODE;
  constexpr int NCI = 2 * (LTS + 1);       // in-tile channels, li = 2 r + k
  constexpr int NTAP = NCI * (TB + 1);
  constexpr int SZR = SH::size(LTS);
  static_assert(NO % NT == 0, "tile must be a multiple of the block");
  static_assert(NTAP + TB * SZR <= NT, "tap and coarse staging threads");
  static_assert(UP <= 2 * NT, "two owned upper nodes per thread");
  static_assert(D == 1 || !MODE || (NT % TS == 0 && EPTO * NT == NO), "column strips");
  __shared__ double s_v[TB * UP];          // upper levels, unpadded, per slab
  __shared__ double s_f[MODE ? TB * L0 : 1];
  __shared__ int s_q[NCI][TB + 1];         // q0 of slabs nb-1 .. nb+TB-1 (-1: none)
  __shared__ double s_w[NCI][TB][3];       // weights of slabs nb .. nb+TB-1
  __shared__ double s_co[TB * SZR];        // coarse-level values at level-A0 nodes

  const Geometry g = A.g;
  const int tid = threadIdx.x;
  int tile, chunk;
  stream_block(lin, (D == 2) ? g.ntile * g.ntile : g.ntile, g.nchunk, tile, chunk);
  const int tx = tile % g.ntile;
  const int ty = (D == 2) ? tile / g.ntile : 0;
  int n0, n1;
  chunk_span(g, chunk, n0, n1);
  const long long nsp = (D == 2) ? (long long)g.nxf * g.nxf : g.nxf;
  const int R = g.R;
  const bool use_coarse = g.A0 > 1 && A.coarse != nullptr;

  // ---- owned upper nodes: coefficient offsets and windows in registers ----
  Owned<D, TS, MODE> own[2];
  own[0].set(tid);
  own[1].set(tid + NT);
  int coff[2];  // offset of the node in a time plane of its level (-1: boundary)
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    coff[i] = -1;
    const int r = own[i].r;
    if (r >= 1 && r <= R) {
      const int a = g.J - r, na = (1 << a) - 1;
      const int Px = tile_lo(TS, tx, r, MODE) + own[i].jx;
      const int Py = (D == 2) ? tile_lo(TS, ty, r, MODE) + own[i].jy : 0;
      if (interior(Px, na) && (D == 1 || interior(Py, na)))
        coff[i] = (Px - 1) + (D == 2 ? (Py - 1) * na : 0);
    }
  }
  // window c[0..2] = coefficients q0..q0+2, c[3] = q0+3 (prefetched)
  double cw[2][2][4];
  int cq[2][2];  // q0 of the current window
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      cq[i][k] = 0;
      cw[i][k][0] = cw[i][k][1] = cw[i][k][2] = cw[i][k][3] = 0.0;
    }
  auto coef = [&](const Channel &C, int q, int off) -> double {
    if (off < 0 || q >= C.nq) return 0.0;
    const int na = (1 << C.a) - 1;
    const long long nspa = (D == 2) ? (long long)na * na : na;
    return C.data[(long long)q * nspa + off];
  };
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = own[i].r;
    if (r < 1 || r > R) continue;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (!C.active) continue;
      const int q = gld(C.q0, n0);
      cq[i][k] = q;
#pragma unroll
      for (int o = 0; o < 4; ++o) cw[i][k][o] = coef(C, q + o, coff[i]);
    }
  }
  // level-J channels keep one time window per chunk (the chunks are cut
  // where it moves): nodes q0(n0) + 0, 1, 2
  const int lo0x = tile_lo(TS, tx, 0, MODE), lo0y = tile_lo(TS, ty, 0, MODE);
  double rc[EPT0][NC0][3];
#pragma unroll
  for (int e = 0; e < EPT0; ++e) {
    const int p = tid + e * NT;
    const int Px = lo0x + p % NF, Py = (D == 2) ? lo0y + p / NF : 0;
    const int off = (p < L0 && interior(Px, g.nxf) && (D == 1 || interior(Py, g.nxf)))
                        ? (Px - 1) + (D == 2 ? (Py - 1) * g.nxf : 0)
                        : -1;
#pragma unroll
    for (int k = 0; k < NC0; ++k) {
      const Channel &C = A.ch[(g.J - 1) * 2 + k];
      rc[e][k][0] = rc[e][k][1] = rc[e][k][2] = 0.0;
      if (!C.active) continue;
      const int qj = gld(C.q0, n0);  // the chunk's window (fixed within the chunk)
#pragma unroll
      for (int o = 0; o < 3; ++o) rc[e][k][o] = coef(C, qj + o, off);
    }
  }
  double basev[EPT0];
#pragma unroll
  for (int e = 0; e < EPT0; ++e) {
    basev[e] = 0.0;
    const int p = tid + e * NT;
    if (!MODE && p < L0 && base != nullptr) {
      const int Px = lo0x + p % NF, Py = (D == 2) ? lo0y + p / NF : 0;
      if (interior(Px, g.nxf) && (D == 1 || interior(Py, g.nxf)))
        basev[e] = base[(D == 2 ? (long long)(Py - 1) * g.nxf : 0) + (Px - 1)];
    }
  }

  // ---- tap entries and coarse values of the next batch (registers) ----
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
  const int co_i = tid - NTAP;
  int co_off = -1, co_s = 0;
  if (use_coarse && co_i >= 0 && co_i < TB * SZR) {
    co_s = co_i / SZR;
    const int j = co_i - co_s * SZR;
    constexpr int nrR = SH::nodes(LTS);
    const int Px = tile_lo(TS, tx, LTS, MODE) + j % nrR;
    const int Py = (D == 2) ? tile_lo(TS, ty, LTS, MODE) + j / nrR : 0;
    const int n0a = (1 << g.A0) - 1;
    if (interior(Px, n0a) && (D == 1 || interior(Py, n0a)))
      co_off = (Px - 1) + (D == 2 ? (Py - 1) * n0a : 0);
  }
  const long long nsp0 = (D == 2) ? (long long)((1 << g.A0) - 1) * ((1 << g.A0) - 1)
                                  : (1 << g.A0) - 1;
  int pq = -1;
  double pw0 = 0.0, pw1 = 0.0, pw2 = 0.0, pco = 0.0;
  // unconditional loads from valid addresses, results selected (see k_restrict)
  const int *tq0 = my_q0 != nullptr ? my_q0 : A.safe_q0;
  const double *tw = my_q0 != nullptr ? my_w : A.safe_w;
  const double *cbase = use_coarse ? A.coarse : A.safe_w;
  auto tap_ok = [&](int nb) {
    const int n = nb - 1 + my_s;
    return my_q0 != nullptr && n >= n0 && n < n1;
  };
  auto co_ok = [&](int nb) { return co_off >= 0 && nb + co_s < n1; };
  auto fetch_taps = [&](int nb) {
    const int nc = tap_ok(nb) ? nb - 1 + my_s : 0;
    pq = tq0[nc];
    pw0 = tw[3 * nc];
    pw1 = tw[3 * nc + 1];
    pw2 = tw[3 * nc + 2];
    pco = cbase[co_ok(nb) ? (long long)(nb + co_s) * nsp0 + co_off : 0];
  };

  fetch_taps(n0);
  for (int nb = n0; nb < n1; nb += TB) {
    const int cnt = min(TB, n1 - nb);
    if (tid < NTAP) {
      const int li = tid / (TB + 1);
      const bool ok = tap_ok(nb);
      s_q[li][my_s] = ok ? pq : -1;
      if (my_s > 0) {
        s_w[li][my_s - 1][0] = ok ? pw0 : 0.0;
        s_w[li][my_s - 1][1] = ok ? pw1 : 0.0;
        s_w[li][my_s - 1][2] = ok ? pw2 : 0.0;
      }
    } else if (co_i < TB * SZR) {
      s_co[co_i] = co_ok(nb) ? pco : 0.0;
    }
    __syncthreads();
    if (nb + TB < n1) fetch_taps(nb + TB);
    // phase A: owners evaluate their node in time (register windows); the
    // level loop is unrolled so that channel fields are wave-uniform
#pragma unroll
    for (int r = 1; r <= LTS; ++r) {
      if (r > R) break;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (own[i].r != r) continue;
        for (int s = 0; s < cnt; ++s) {
          double v = (r == R && use_coarse) ? s_co[s * SZR + own[i].j] : 0.0;
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
            if (!C.active) continue;
            const int li = 2 * r + k;
            if (s_q[li][s + 1] > cq[i][k]) {  // advance by one time index
              cq[i][k] += 1;
              cw[i][k][0] = cw[i][k][1];
              cw[i][k][1] = cw[i][k][2];
              cw[i][k][2] = cw[i][k][3];
              cw[i][k][3] = coef(C, cq[i][k] + 3, coff[i]);
            }
            v += C.scale * (s_w[li][s][0] * cw[i][k][0] + s_w[li][s][1] * cw[i][k][1] +
                            s_w[li][s][2] * cw[i][k][2]);
          }
          s_v[s * UP + SH::offset(r) - SH::size(0) + own[i].j] = v;
        }
      }
    }
    __syncthreads();
    // phase B: top-down interpolation r = R-1 .. 1 (owners of level r)
#pragma unroll
    for (int r = LTS - 1; r >= 1; --r) {
      if (r >= R) continue;
      const int nr = SH::nodes(r), pn = SH::nodes(r + 1);
      const int lox = tile_lo(TS, tx, r, MODE), loy = tile_lo(TS, ty, r, MODE);
      const int plox = tile_lo(TS, tx, r + 1, MODE), ploy = tile_lo(TS, ty, r + 1, MODE);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (own[i].r != r) continue;
        const int Px = lox + own[i].jx, Py = (D == 2) ? loy + own[i].jy : 0;
        const int xl = (Px >> 1) - plox, xh = ((Px + 1) >> 1) - plox;
        const int yl = (D == 2) ? (Py >> 1) - ploy : 0, yh = (D == 2) ? ((Py + 1) >> 1) - ploy : 0;
        for (int s = 0; s < cnt; ++s) {
          const double *par = s_v + s * UP + SH::offset(r + 1) - SH::size(0);
          const double add = (D == 1) ? 0.5 * (par[xl] + par[xh])
                                      : 0.25 * (par[yl * pn + xl] + par[yl * pn + xh] +
                                                par[yh * pn + xl] + par[yh * pn + xh]);
          s_v[s * UP + SH::offset(r) - SH::size(0) + own[i].j] += add;
        }
        (void)nr;
      }
      __syncthreads();
    }
    // phase C: fine nodes
    for (int s = 0; s < cnt; ++s) {
      const int n = nb + s;
      double tv[EPT0];
#pragma unroll
      for (int e = 0; e < EPT0; ++e) tv[e] = 0.0;
#pragma unroll
      for (int k = 0; k < NC0; ++k) {
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
          if (A.accumulate) o += out[off];
          out[off] = o;
        }
      }
    }
    if (MODE) {
      __syncthreads();
      // mass stencil on the tile (separable; 2-D threads own column strips)
      const int fx = (D == 2) ? tid % TS : tid;
      const int fy0 = (D == 2) ? (tid / TS) * EPTO : 0;
      for (int s = 0; s < cnt; ++s) {
        const int n = nb + s;
        const double *f = s_f + s * L0;
        double o[EPTO];
        if (D == 1) {
          o[0] = A.sx * (f[fx] + f[fx + 2] + 4.0 * f[fx + 1]);
        } else {
          double h[EPTO + 2];
#pragma unroll
          for (int i2 = 0; i2 < EPTO + 2; ++i2) {
            const double *row = f + (fy0 + i2) * NF + fx;
            h[i2] = row[0] + row[2] + 4.0 * row[1];
          }
          const double sxy = A.sx * A.sy;
#pragma unroll
          for (int e = 0; e < EPTO; ++e) o[e] = sxy * (h[e] + h[e + 2] + 4.0 * h[e + 1]);
        }
#pragma unroll
        for (int e = 0; e < EPTO; ++e) {
          const int Px = TS * tx + fx, Py = (D == 2) ? TS * ty + fy0 + e : 0;
          if (!interior(Px, g.nxf) || (D == 2 && !interior(Py, g.nxf))) continue;
          const long long off = (long long)n * nsp +
                                (D == 2 ? (long long)(Py - 1) * g.nxf : 0) + (Px - 1);
          double val = o[e];
          if (base != nullptr) val += base[off - (long long)n * nsp];
          if (A.accumulate) val += out[off];
          out[off] = val;
        }
      }
    }
    __syncthreads();
  }
}

template <int D, int TS, int TB, int NT, int MODE, int NC0>
__global__ void __launch_bounds__(NT, SG_WPE) k_prolong(const ProlongArgs A) {
  prolong_body<D, TS, TB, NT, MODE, NC0>(A, A.base, A.out, block_lin());
}

// 2-D prolongation (no stencil) with one 16 x 16 tile per wave: the
// counterpart of k_restrict_w, four tiles side by side per workgroup (rows
// of 64 contiguous outputs per workgroup: fewer cache lines shared with
// other workgroups than a 2 x 2 block) and no workgroup barrier in the slab
// loop.  Per slab: (A) the owners of the tile's
// upper-level nodes evaluate their channels in time (register windows of
// coefficients; the top level adds the levels below the tile from
// A.coarse), (B) top-down interpolation through the levels, (C) the fine
// nodes add their level-J channel and the interpolated level-1 values and
// are written.  Lane l takes column l % 16, rows 4 (l / 16) .. +3, which
// share three level-1 rows; every store instruction writes four whole
// 128-byte rows.  Taps (weights times
// channel sign, and where the window moves on) come from a per-pass host
// table.  The prolongation through the mass stencil is k_prolong_wm.
#ifndef SG_WPEP
#define SG_WPEP 3
#endif
__device__ __forceinline__ void prolong_w_body(const ProlongArgs &A, const double *__restrict__ base,
                                               double *__restrict__ out, int lin) {
  constexpr int TS = 16, LTS = 4;
  using SH = Shape<2, TS, 0>;
  constexpr int L0 = TS * TS;
  constexpr int EF = L0 / 64;             // fine nodes per lane
  constexpr int UP = SH::upper;
  constexpr int NS = (UP + 63) / 64;      // owned upper-node slots per lane
  constexpr int NCI = 2 * (LTS + 1);
  static_assert(NS == 2 && L0 % 64 == 0, "tile shape");
  __shared__ double s_v_w[4][UP];
  __shared__ __align__(16) double s_t_w[4][4 * NCI];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *s_v = s_v_w[wave];
  double *s_t = s_t_w[wave];

  const Geometry g = A.g;
  const int nt = g.ntile, ngx = (nt + 3) >> 2;
  int grp, chunk;
  stream_block(lin, ngx * nt, g.nchunk, grp, chunk);
  const int tx = 4 * (grp % ngx) + wave, ty = grp / ngx;
  if (tx >= nt || ty >= nt) return;  // no workgroup barrier below
  int n0, n1;
  chunk_span(g, chunk, n0, n1);
  const long long nsp = (long long)g.nxf * g.nxf;
  const int R = g.R;
  const bool use_coarse = g.A0 > 1 && A.coarse != nullptr;
  const int n0a = (1 << g.A0) - 1;
  const long long nsp0 = (long long)n0a * n0a;

  // ---- owned upper nodes: coefficient offsets and windows ----
  Owned<2, TS, 0> own[NS];
  int coff[NS], cof0[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    own[i].set(lane + 64 * i);
    coff[i] = -1;
    cof0[i] = -1;
    const int r = own[i].r;
    if (r >= 1 && r <= R) {
      const int na = (1 << (g.J - r)) - 1;
      const int Px = tile_lo(TS, tx, r, 0) + own[i].jx;
      const int Py = tile_lo(TS, ty, r, 0) + own[i].jy;
      if (interior(Px, na) && interior(Py, na)) coff[i] = (Px - 1) + (Py - 1) * na;
      if (r == R && use_coarse && interior(Px, n0a) && interior(Py, n0a))
        cof0[i] = (Px - 1) + (Py - 1) * n0a;
    }
  }
  auto coef = [&](const Channel &C, int q, int off) -> double {
    if (off < 0 || q >= C.nq) return 0.0;
    const int na = (1 << C.a) - 1;
    return (C.data + (long long)q * na * na)[lane_off(off)];
  };
  // coefficient windows q0 .. q0+2 of the owned nodes
  double cw[NS][2][3];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      cw[i][k][0] = cw[i][k][1] = cw[i][k][2] = 0.0;
      const int r = own[i].r;
      if (r < 1 || r > R) continue;
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (!C.active) continue;
      const int q = ld_const(C.q0, n0);
#pragma unroll
      for (int o = 0; o < 3; ++o) cw[i][k][o] = coef(C, q + o, coff[i]);
    }

  // ---- fine nodes: lane = column fx, rows fy0 .. fy0+3; level-J channel
  // (one time window per chunk) and base ----
  const int fx = lane & 15, fy0 = (lane >> 4) * EF;
  const Channel &CJ = A.ch[(g.J - 1) * 2];
  // the chunk's time window of the level-J channel (fixed within the chunk)
  const int qj = CJ.active ? ld_const(CJ.q0, n0) : 0;
  const int Px = TS * tx + fx;
  double rc[EF][3], basev[EF];
#pragma unroll
  for (int e = 0; e < EF; ++e) {
    const int Py = TS * ty + fy0 + e;
    const int off = interior(Px, g.nxf) && interior(Py, g.nxf) ? (Px - 1) + (Py - 1) * g.nxf : -1;
#pragma unroll
    for (int o = 0; o < 3; ++o) rc[e][o] = CJ.active ? coef(CJ, qj + o, off) : 0.0;
    basev[e] = (base != nullptr && off >= 0) ? base[off] : 0.0;
  }
  // coarse values of the next slab (unconditional loads from valid addresses)
  const double *cbase = use_coarse ? A.coarse : A.safe_w;
  double pco[NS];
  auto fetch_co = [&](int n) {
    const double *row = cbase + (use_coarse ? (long long)n * nsp0 : 0);
#pragma unroll
    for (int i = 0; i < NS; ++i) pco[i] = row[lane_off(max(cof0[i], 0))];
  };
  const int pn1 = SH::nodes(1);
  const int plox = tile_lo(TS, tx, 1, 0), ploy = tile_lo(TS, ty, 1, 0);

  // LDS slot of an owned node and the offset of its level's tap entries
  int sidx[NS], tslot[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int r = own[i].r;
    const bool act = r >= 1 && r <= R;
    sidx[i] = act ? SH::offset(r) - SH::size(0) + own[i].j : -1;
    tslot[i] = act ? 8 * r : 0;
  }
  SlabTaps<NCI> tp;
  tp.fetch(A.taps, n0, lane);

  // the coarse values and taps of slab n + 1 are taken over at the end of
  // slab n, before its stores: loads and stores share one completion counter,
  // so a store issued just before a wait for loads would hold that wait up
  double co[NS];
  auto take_next = [&]() {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      co[i] = cof0[i] >= 0 ? pco[i] : 0.0;
      take(co[i]);
    }
    tp.stage(s_t, lane);
  };
  fetch_co(n0);
  take_next();
  for (int n = n0; n < n1; ++n) {
    const TapEntry *tn = A.taps + (long long)n * NCI;
    if (n + 1 < n1) {
      fetch_co(n + 1);
      tp.fetch(A.taps, n + 1, lane);
    }
    wave_sync();
    // (A) owners evaluate their node in time: windows that move on at this
    // slab shift first, then every slot applies the taps of its own level
    const int mv = slab_moves(s_t);
    if (mv != 0) {
#pragma unroll
      for (int r = 1; r <= LTS; ++r) {
        if (r > R) break;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          if (!((mv >> (2 * r + k)) & 1)) continue;
          const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
          const int q = (int)ld_const(tn, 2 * r + k).base;  // new first time index
#pragma unroll
          for (int i = 0; i < NS; ++i) {
            if (own[i].r != r) continue;
            cw[i][k][0] = cw[i][k][1];
            cw[i][k][1] = cw[i][k][2];
            cw[i][k][2] = coef(C, q + 2, coff[i]);
            take(cw[i][k][2]);  // waited for here, on the rare path
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const double *t = s_t + tslot[i];
      const double2 a0 = *reinterpret_cast<const double2 *>(t);
      const double2 a1 = *reinterpret_cast<const double2 *>(t + 2);
      const double2 b0 = *reinterpret_cast<const double2 *>(t + 4);
      const double2 b1 = *reinterpret_cast<const double2 *>(t + 6);
      const double v = co[i] + a0.x * cw[i][0][0] + a0.y * cw[i][0][1] + a1.x * cw[i][0][2] +
                       b0.x * cw[i][1][0] + b0.y * cw[i][1][1] + b1.x * cw[i][1][2];
      if (sidx[i] >= 0) s_v[sidx[i]] = v;
    }
    // (B) top-down interpolation r = R-1 .. 1
#pragma unroll
    for (int r = LTS - 1; r >= 1; --r) {
      if (r >= R) continue;
      wave_sync();
      const int pn = SH::nodes(r + 1);
      const int lox = tile_lo(TS, tx, r, 0), loy = tile_lo(TS, ty, r, 0);
      const int qx = tile_lo(TS, tx, r + 1, 0), qy = tile_lo(TS, ty, r + 1, 0);
      const double *par = s_v + SH::offset(r + 1) - SH::size(0);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        if (own[i].r != r) continue;
        const int Px = lox + own[i].jx, Py = loy + own[i].jy;
        const int xl = (Px >> 1) - qx, xh = ((Px + 1) >> 1) - qx;
        const int yl = (Py >> 1) - qy, yh = ((Py + 1) >> 1) - qy;
        s_v[SH::offset(r) - SH::size(0) + own[i].j] +=
            0.25 * (par[yl * pn + xl] + par[yl * pn + xh] + par[yh * pn + xl] + par[yh * pn + xh]);
      }
    }
    wave_sync();
    // (C) fine nodes: bilinear interpolation from level 1, x first; the
    // lane's rows fy0 .. fy0+3 (fy0 even) use level-1 rows r0 .. r0+2
    const double2 tj01 = *reinterpret_cast<const double2 *>(s_t);  // level-J channel
    const double tj2 = s_t[2];
    if (n + 1 < n1) take_next();  // before this slab's stores
    wave_sync();
    double xs[3] = {0.0, 0.0, 0.0};
    if (R >= 1) {
      const int kx = (Px >> 1) - plox, r0 = ((TS * ty + fy0) >> 1) - ploy;
      const double wx1 = (Px & 1) ? 0.5 : 0.0, wx0 = 1.0 - wx1;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double *zr = s_v + (r0 + r) * pn1 + kx;
        xs[r] = wx0 * zr[0] + wx1 * zr[1];
      }
    }
    const double lev[EF] = {xs[0], 0.5 * (xs[0] + xs[1]), xs[1], 0.5 * (xs[1] + xs[2])};
#pragma unroll
    for (int e = 0; e < EF; ++e) {
      const int Py = TS * ty + fy0 + e;
      const double v = tj01.x * rc[e][0] + tj01.y * rc[e][1] + tj2 * rc[e][2] + lev[e];
      if (interior(Px, g.nxf) && interior(Py, g.nxf)) {
        const long long off = (long long)n * nsp + (long long)(Py - 1) * g.nxf + (Px - 1);
        double o = v + basev[e];
        if (A.accumulate) o += out[off];
        out[off] = o;
      }
    }
  }
}

__global__ void __launch_bounds__(256, SG_WPEP) k_prolong_w(const ProlongArgs A) {
  prolong_w_body(A, A.base, A.out, block_lin());
}

// 2-D prolongation through the fine mass stencil, one 16 x 16 output tile
// per wave.  The upper levels are evaluated and interpolated as in
// k_prolong_w, on a region with one more node on each side.  The fine values
// themselves are never formed: with F = Phi_1 z + (level-J channel), the
// mass stencil of the interpolant is, per axis, a fixed stencil on level 1
// (P1 hats, fine spacing h): at an even fine node 2K it is
// h/12 (z_{K-1} + 10 z_K + z_{K+1}), at an odd node 2K+1 it is
// h/2 (z_K + z_{K+1}); the 2-D stencil is the tensor product.  The mass
// stencil of the level-J channel's three coefficient fields is applied once,
// before the slab loop, and kept in LDS.  Lane l writes column l % 16, rows
// 4 (l / 16) .. +3, which share four level-1 rows.  Three workgroups per CU:
// at four the register budget of 128 spilled the coefficient windows.
#ifndef SG_WPEM
#define SG_WPEM 3
#endif
__device__ __forceinline__ void prolong_wm_body(const ProlongArgs &A, const double *__restrict__ base,
                                                double *__restrict__ out, int lin) {
  constexpr int TS = 16, LTS = 4;
  using SH = Shape<2, TS, 1>;
  constexpr int NF = TS + 2;              // fine region with its ring (setup only)
  constexpr int L0 = NF * NF;
  constexpr int EF = (L0 + 63) / 64;
  constexpr int UP = SH::upper;
  constexpr int NS = (UP + 63) / 64;      // owned upper-node slots per lane
  constexpr int NCI = 2 * (LTS + 1);
  constexpr int NO = TS * TS / 64;        // outputs per lane
  static_assert(NS == 3 && NO == 4, "tile shape");
  __shared__ double s_v_w[4][UP];
  __shared__ double s_f_w[4][L0];
  __shared__ double s_m_w[4][3][TS * TS];  // mass stencil of the level-J coefficients
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *s_v = s_v_w[wave];
  double *s_f = s_f_w[wave];
  double (*s_m)[TS * TS] = s_m_w[wave];
  double *s_t = s_f;  // the slab taps reuse the set-up region

  const Geometry g = A.g;
  const int nt = g.ntile, ngx = (nt + 3) >> 2;
  int grp, chunk;
  stream_block(lin, ngx * nt, g.nchunk, grp, chunk);
  const int tx = 4 * (grp % ngx) + wave, ty = grp / ngx;
  if (tx >= nt || ty >= nt) return;  // no workgroup barrier below
  int n0, n1;
  chunk_span(g, chunk, n0, n1);
  const long long nsp = (long long)g.nxf * g.nxf;
  const int R = g.R;
  const bool use_coarse = g.A0 > 1 && A.coarse != nullptr;
  const int n0a = (1 << g.A0) - 1;
  const long long nsp0 = (long long)n0a * n0a;
  const double hx = 6.0 * A.sx, hy = 6.0 * A.sy;  // fine mesh widths

  // ---- owned upper nodes: coefficient offsets and windows ----
  Owned<2, TS, 1> own[NS];
  int coff[NS], cof0[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    own[i].set(lane + 64 * i);
    coff[i] = -1;
    cof0[i] = -1;
    const int r = own[i].r;
    if (r >= 1 && r <= R) {
      const int na = (1 << (g.J - r)) - 1;
      const int Px = tile_lo(TS, tx, r, 1) + own[i].jx;
      const int Py = tile_lo(TS, ty, r, 1) + own[i].jy;
      if (interior(Px, na) && interior(Py, na)) coff[i] = (Px - 1) + (Py - 1) * na;
      if (r == R && use_coarse && interior(Px, n0a) && interior(Py, n0a))
        cof0[i] = (Px - 1) + (Py - 1) * n0a;
    }
  }
  auto coef = [&](const Channel &C, int q, int off) -> double {
    if (off < 0 || q >= C.nq) return 0.0;
    const int na = (1 << C.a) - 1;
    return (C.data + (long long)q * na * na)[lane_off(off)];
  };
  double cw[NS][2][3];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      cw[i][k][0] = cw[i][k][1] = cw[i][k][2] = 0.0;
      const int r = own[i].r;
      if (r < 1 || r > R) continue;
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (!C.active) continue;
      const int q = ld_const(C.q0, n0);
#pragma unroll
      for (int o = 0; o < 3; ++o) cw[i][k][o] = coef(C, q + o, coff[i]);
    }

  // ---- outputs of this lane and the mass stencil of the level-J channel ----
  const int fx = lane & 15, fy0 = (lane >> 4) * NO;
  const int lo0x = tile_lo(TS, tx, 0, 1), lo0y = tile_lo(TS, ty, 0, 1);
  const Channel &CJ = A.ch[(g.J - 1) * 2];
  // the chunk's time window of the level-J channel (fixed within the chunk)
  const int qj = CJ.active ? ld_const(CJ.q0, n0) : 0;
#pragma unroll
  for (int o = 0; o < 3; ++o) {
#pragma unroll
    for (int e = 0; e < EF; ++e) {
      const int p = lane + 64 * e;
      if (p >= L0) continue;
      const int Px = lo0x + p % NF, Py = lo0y + p / NF;
      const int off = interior(Px, g.nxf) && interior(Py, g.nxf) ? (Px - 1) + (Py - 1) * g.nxf : -1;
      s_f[p] = CJ.active ? coef(CJ, qj + o, off) : 0.0;
    }
    wave_sync();
#pragma unroll
    for (int e = 0; e < NO; ++e) {
      double h[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double *row = s_f + (fy0 + e + i) * NF + fx;
        h[i] = row[0] + row[2] + 4.0 * row[1];
      }
      s_m[o][(fy0 + e) * TS + fx] = A.sx * A.sy * (h[0] + h[2] + 4.0 * h[1]);
    }
    wave_sync();
  }
  // level-1 stencil of the lane's outputs: x taps (level-1 column, weight)
  // for column Px = 16 tx + fx, y taps for rows Py = 16 ty + fy0 + e
  const int pn1 = SH::nodes(1);
  const int plox = tile_lo(TS, tx, 1, 1), ploy = tile_lo(TS, ty, 1, 1);
  const int Pxo = TS * tx + fx;
  const bool xin = interior(Pxo, g.nxf);
  const int kx = (Pxo >> 1) - plox;
  const bool xeven = (Pxo & 1) == 0;
  // even: columns kx-1, kx, kx+1 with h/12 (1, 10, 1); odd: kx, kx+1 with h/2
  const int cx0 = xeven ? kx - 1 : kx;
  const double wx0 = xeven ? hx / 12.0 : 0.5 * hx, wx1 = xeven ? 10.0 * hx / 12.0 : 0.5 * hx,
               wx2 = xeven ? hx / 12.0 : 0.0;
  const double *cbase = use_coarse ? A.coarse : A.safe_w;
  double pco[NS];
  auto fetch_co = [&](int n) {
    const double *row = cbase + (use_coarse ? (long long)n * nsp0 : 0);
#pragma unroll
    for (int i = 0; i < NS; ++i) pco[i] = row[lane_off(max(cof0[i], 0))];
  };

  // LDS slot of an owned node and the offset of its level's tap entries
  int sidx[NS], tslot[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int r = own[i].r;
    const bool act = r >= 1 && r <= R;
    sidx[i] = act ? SH::offset(r) - SH::size(0) + own[i].j : -1;
    tslot[i] = act ? 8 * r : 0;
  }
  SlabTaps<NCI> tp;
  tp.fetch(A.taps, n0, lane);

  // the coarse values and taps of slab n + 1 are taken over at the end of
  // slab n, before its stores: loads and stores share one completion counter,
  // so a store issued just before a wait for loads would hold that wait up
  double co[NS];
  auto take_next = [&]() {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      co[i] = cof0[i] >= 0 ? pco[i] : 0.0;
      take(co[i]);
    }
    tp.stage(s_t, lane);
  };
  fetch_co(n0);
  take_next();
  for (int n = n0; n < n1; ++n) {
    const TapEntry *tn = A.taps + (long long)n * NCI;
    if (n + 1 < n1) {
      fetch_co(n + 1);
      tp.fetch(A.taps, n + 1, lane);
    }
    wave_sync();
    // (A) owners evaluate their node in time: windows that move on at this
    // slab shift first, then every slot applies the taps of its own level
    const int mv = slab_moves(s_t);
    if (mv != 0) {
#pragma unroll
      for (int r = 1; r <= LTS; ++r) {
        if (r > R) break;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          if (!((mv >> (2 * r + k)) & 1)) continue;
          const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
          const int q = (int)ld_const(tn, 2 * r + k).base;  // new first time index
#pragma unroll
          for (int i = 0; i < NS; ++i) {
            if (own[i].r != r) continue;
            cw[i][k][0] = cw[i][k][1];
            cw[i][k][1] = cw[i][k][2];
            cw[i][k][2] = coef(C, q + 2, coff[i]);
            take(cw[i][k][2]);  // waited for here, on the rare path
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const double *t = s_t + tslot[i];
      const double2 a0 = *reinterpret_cast<const double2 *>(t);
      const double2 a1 = *reinterpret_cast<const double2 *>(t + 2);
      const double2 b0 = *reinterpret_cast<const double2 *>(t + 4);
      const double2 b1 = *reinterpret_cast<const double2 *>(t + 6);
      const double v = co[i] + a0.x * cw[i][0][0] + a0.y * cw[i][0][1] + a1.x * cw[i][0][2] +
                       b0.x * cw[i][1][0] + b0.y * cw[i][1][1] + b1.x * cw[i][1][2];
      if (sidx[i] >= 0) s_v[sidx[i]] = v;
    }
    // (B) top-down interpolation r = R-1 .. 1
#pragma unroll
    for (int r = LTS - 1; r >= 1; --r) {
      if (r >= R) continue;
      wave_sync();
      const int pn = SH::nodes(r + 1);
      const int lox = tile_lo(TS, tx, r, 1), loy = tile_lo(TS, ty, r, 1);
      const int qx = tile_lo(TS, tx, r + 1, 1), qy = tile_lo(TS, ty, r + 1, 1);
      const double *par = s_v + SH::offset(r + 1) - SH::size(0);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        if (own[i].r != r) continue;
        const int Px = lox + own[i].jx, Py = loy + own[i].jy;
        const int xl = (Px >> 1) - qx, xh = ((Px + 1) >> 1) - qx;
        const int yl = (Py >> 1) - qy, yh = ((Py + 1) >> 1) - qy;
        s_v[SH::offset(r) - SH::size(0) + own[i].j] +=
            0.25 * (par[yl * pn + xl] + par[yl * pn + xh] + par[yh * pn + xl] + par[yh * pn + xh]);
      }
    }
    wave_sync();
    // (C) outputs: level-1 stencil plus the level-J channel.  The lane's
    // four rows Py0 .. Py0+3 (Py0 even) use level-1 rows K0-1 .. K0+2,
    // K0 = Py0 / 2; each row is first reduced with the x stencil.
    const double2 tj01 = *reinterpret_cast<const double2 *>(s_t);  // level-J channel
    const double tj2 = s_t[2];
    if (n + 1 < n1) take_next();  // before this slab's stores
    wave_sync();
    double xs[4] = {0.0, 0.0, 0.0, 0.0};
    if (R >= 1) {
      const int r0 = ((TS * ty + fy0) >> 1) - ploy - 1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double *zr = s_v + (r0 + r) * pn1;
        xs[r] = wx0 * zr[cx0] + wx1 * zr[cx0 + 1] + wx2 * zr[min(cx0 + 2, pn1 - 1)];
      }
    }
    const double ye = hy / 12.0, yo = 0.5 * hy;
    const double lev[4] = {ye * (xs[0] + 10.0 * xs[1] + xs[2]), yo * (xs[1] + xs[2]),
                           ye * (xs[1] + 10.0 * xs[2] + xs[3]), yo * (xs[2] + xs[3])};
#pragma unroll
    for (int e = 0; e < NO; ++e) {
      const int Py = TS * ty + fy0 + e;
      const int po = (fy0 + e) * TS + fx;
      double val = tj01.x * s_m[0][po] + tj01.y * s_m[1][po] + tj2 * s_m[2][po] + lev[e];
      if (xin && interior(Py, g.nxf)) {
        const long long off = (long long)n * nsp + (long long)(Py - 1) * g.nxf + (Pxo - 1);
        if (base != nullptr) val += base[off - (long long)n * nsp];
        if (A.accumulate) val += out[off];
        out[off] = val;
      }
    }
  }
}

__global__ void __launch_bounds__(256, SG_WPEM) k_prolong_wm(const ProlongArgs A) {
  prolong_wm_body(A, A.base, A.out, block_lin());
}

// Energy of u_h at given instants (2-D, 16 x 16 tiles), without forming the
// fields in memory: per wave one tile and a chunk of instants.  Per instant
// the tile's upper-level nodes are evaluated in time twice over the same
// coefficient windows, with the value taps of A.taps and the derivative taps
// of taps_d (and the levels below the tile from A.coarse and coarse_d), both
// fields are interpolated down to level 1, and the values of u_h (plus u0 =
// A.base) and d_t u_h at the tile's 17 x 17 nodes (its own 16 x 16 and the
// first row and column of the next tiles, which close its elements) go to
// LDS.  Each lane then applies the Q1 element mass form to d_t u_h and the
// c^2-weighted stiffness form to u_h on its four elements (lower-left nodes
// in column l % 16, rows 4 (l / 16) .. +3), and the wave's sum in a fixed
// order is part[n][tile].  Two workgroups per CU: both fields' windows, taps
// and level-J coefficients stay in registers.
__global__ void __launch_bounds__(256, 2) k_energy_w(const ProlongArgs A,
                                                          const TapEntry *__restrict__ taps_d,
                                                          const double *__restrict__ coarse_d,
                                                          const double *__restrict__ ce,
                                                          double hx, double hy,
                                                          double *__restrict__ part) {
  constexpr int TS = 16, LTS = 4, NP = TS + 1;
  using SH = Shape<2, TS, 0>;
  constexpr int EF = TS * TS / 64;       // own nodes (and elements) per lane
  constexpr int UP = SH::upper;
  constexpr int NS = (UP + 63) / 64;     // owned upper-node slots per lane
  constexpr int NCI = 2 * (LTS + 1);
  constexpr int NRING = 2 * TS + 1;      // column 16 (rows 0..16), row 16 (columns 0..15)
  static_assert(NS == 2 && NRING <= 64, "tile shape");
  __shared__ double s_v_w[4][2][UP];
  __shared__ __align__(16) double s_t_w[4][2][4 * NCI];
  __shared__ double s_f_w[4][2][NP * NP];
  // the lanes' element sums of up to RB instants, one padded row per instant
  // (pitch RP: 16-byte rows that fall on different banks)
  constexpr int RB = 16, RP = 66;
  __shared__ __align__(16) double s_r_w[4][RB * RP];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *s_v[2] = {s_v_w[wave][0], s_v_w[wave][1]};  // value, derivative
  double *s_t[2] = {s_t_w[wave][0], s_t_w[wave][1]};
  double *s_f[2] = {s_f_w[wave][0], s_f_w[wave][1]};

  const Geometry g = A.g;
  const int nt = g.ntile, ngx = (nt + 3) >> 2;
  int grp, chunk;
  stream_block(block_lin(), ngx * nt, g.nchunk, grp, chunk);
  const int tx = 4 * (grp % ngx) + wave, ty = grp / ngx;
  if (tx >= nt || ty >= nt) return;  // no workgroup barrier below
  const int tile = ty * nt + tx, ntileD = nt * nt;
  int n0, n1;
  chunk_span(g, chunk, n0, n1);
  const int R = g.R;
  const int N = g.nxf + 1;  // elements per axis
  const bool use_coarse = g.A0 > 1 && A.coarse != nullptr;
  const int n0a = (1 << g.A0) - 1;
  const long long nsp0 = (long long)n0a * n0a;

  // ---- owned upper nodes: coefficient offsets and windows (shared by both
  // fields: the value and derivative taps have the same windows) ----
  Owned<2, TS, 0> own[NS];
  int coff[NS], cof0[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    own[i].set(lane + 64 * i);
    coff[i] = -1;
    cof0[i] = -1;
    const int r = own[i].r;
    if (r >= 1 && r <= R) {
      const int na = (1 << (g.J - r)) - 1;
      const int Px = tile_lo(TS, tx, r, 0) + own[i].jx;
      const int Py = tile_lo(TS, ty, r, 0) + own[i].jy;
      if (interior(Px, na) && interior(Py, na)) coff[i] = (Px - 1) + (Py - 1) * na;
      if (r == R && use_coarse && interior(Px, n0a) && interior(Py, n0a))
        cof0[i] = (Px - 1) + (Py - 1) * n0a;
    }
  }
  auto coef = [&](const Channel &C, int q, int off) -> double {
    if (off < 0 || q >= C.nq) return 0.0;
    const int na = (1 << C.a) - 1;
    return (C.data + (long long)q * na * na)[lane_off(off)];
  };
  double cw[NS][2][3];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      cw[i][k][0] = cw[i][k][1] = cw[i][k][2] = 0.0;
      const int r = own[i].r;
      if (r < 1 || r > R) continue;
      const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
      if (!C.active) continue;
      const int q = ld_const(C.q0, n0);
#pragma unroll
      for (int o = 0; o < 3; ++o) cw[i][k][o] = coef(C, q + o, coff[i]);
    }

  // ---- the lane's nodes: own column fx, rows fy0 .. fy0+3; ring node
  // lane < 33: (16, lane) for lane <= 16, else (lane - 17, 16).  Level-J
  // channel coefficients (one time window per chunk) and u0 at each ----
  const int fx = lane & 15, fy0 = (lane >> 4) * EF;
  const bool has_ring = lane < NRING;
  const int rx = lane <= TS ? TS : lane - (TS + 1), ry = lane <= TS ? lane : TS;
  const Channel &CJ = A.ch[(g.J - 1) * 2];
  // the chunk's time window of the level-J channel (fixed within the chunk)
  const int qj = CJ.active ? ld_const(CJ.q0, n0) : 0;
  double rc[EF + 1][3], basev[EF + 1];
#pragma unroll
  for (int e = 0; e <= EF; ++e) {
    const int x = e < EF ? fx : rx, y = e < EF ? fy0 + e : ry;
    const int Px = TS * tx + x, Py = TS * ty + y;
    const bool in = (e < EF || has_ring) && interior(Px, g.nxf) && interior(Py, g.nxf);
    const int off = in ? (Px - 1) + (Py - 1) * g.nxf : -1;
#pragma unroll
    for (int o = 0; o < 3; ++o) rc[e][o] = CJ.active ? coef(CJ, qj + o, off) : 0.0;
    basev[e] = (A.base != nullptr && off >= 0) ? A.base[off] : 0.0;
  }
  // c^2 of the lane's elements (lower-left nodes (fx, fy0 + e)); zero for
  // elements outside the domain
  double c2e[EF];
#pragma unroll
  for (int e = 0; e < EF; ++e) {
    const int ex = TS * tx + fx, ey = TS * ty + fy0 + e;
    c2e[e] = (ex < N && ey < N) ? ce[(long long)ey * N + ex] : 0.0;
  }
  const double *cbase[2] = {use_coarse ? A.coarse : A.safe_w, use_coarse ? coarse_d : A.safe_w};
  double pco[2][NS];
  auto fetch_co = [&](int n) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const double *row = cbase[f] + (use_coarse ? (long long)n * nsp0 : 0);
#pragma unroll
      for (int i = 0; i < NS; ++i) pco[f][i] = row[lane_off(max(cof0[i], 0))];
    }
  };
  const int pn1 = SH::nodes(1);

  int sidx[NS], tslot[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int r = own[i].r;
    const bool act = r >= 1 && r <= R;
    sidx[i] = act ? SH::offset(r) - SH::size(0) + own[i].j : -1;
    tslot[i] = act ? 8 * r : 0;
  }
  SlabTaps<NCI> tp[2];
  tp[0].fetch(A.taps, n0, lane);
  tp[1].fetch(taps_d, n0, lane);

  double co[2][NS];
  auto take_next = [&]() {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        co[f][i] = cof0[i] >= 0 ? pco[f][i] : 0.0;
        take(co[f][i]);
      }
      tp[f].stage(s_t[f], lane);
    }
  };
  // level-1 part of a field at the tile's node (x, y), 0 <= x, y <= 16
  auto lev1 = [&](const double *v1, int x, int y) -> double {
    const int kx = x >> 1, ky = y >> 1;
    const bool ox = x & 1, oy = y & 1;
    const double a = v1[ky * pn1 + kx], b = ox ? v1[ky * pn1 + kx + 1] : a;
    const double r0 = ox ? 0.5 * (a + b) : a;
    if (!oy) return r0;
    const double c = v1[(ky + 1) * pn1 + kx], d = ox ? v1[(ky + 1) * pn1 + kx + 1] : c;
    const double r1 = ox ? 0.5 * (c + d) : c;
    return 0.5 * (r0 + r1);
  };
  fetch_co(n0);
  take_next();
  for (int n = n0; n < n1; ++n) {
    const TapEntry *tn = A.taps + (long long)n * NCI;
    if (n + 1 < n1) {
      fetch_co(n + 1);
      tp[0].fetch(A.taps, n + 1, lane);
      tp[1].fetch(taps_d, n + 1, lane);
    }
    wave_sync();
    // (A) windows that move on at this slab shift first (the same for both
    // fields), then every slot applies the taps of its own level
    const int mv = slab_moves(s_t[0]);
    if (mv != 0) {
#pragma unroll
      for (int r = 1; r <= LTS; ++r) {
        if (r > R) break;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          if (!((mv >> (2 * r + k)) & 1)) continue;
          const Channel &C = A.ch[(g.J - r - 1) * 2 + k];
          const int q = (int)ld_const(tn, 2 * r + k).base;  // new first time index
#pragma unroll
          for (int i = 0; i < NS; ++i) {
            if (own[i].r != r) continue;
            cw[i][k][0] = cw[i][k][1];
            cw[i][k][1] = cw[i][k][2];
            cw[i][k][2] = coef(C, q + 2, coff[i]);
            take(cw[i][k][2]);
          }
        }
      }
    }
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const double *t = s_t[f] + tslot[i];
        const double2 a0 = *reinterpret_cast<const double2 *>(t);
        const double2 a1 = *reinterpret_cast<const double2 *>(t + 2);
        const double2 b0 = *reinterpret_cast<const double2 *>(t + 4);
        const double2 b1 = *reinterpret_cast<const double2 *>(t + 6);
        const double v = co[f][i] + a0.x * cw[i][0][0] + a0.y * cw[i][0][1] + a1.x * cw[i][0][2] +
                         b0.x * cw[i][1][0] + b0.y * cw[i][1][1] + b1.x * cw[i][1][2];
        if (sidx[i] >= 0) s_v[f][sidx[i]] = v;
      }
    // (B) top-down interpolation r = R-1 .. 1, both fields
#pragma unroll
    for (int r = LTS - 1; r >= 1; --r) {
      if (r >= R) continue;
      wave_sync();
      const int pn = SH::nodes(r + 1);
      const int lox = tile_lo(TS, tx, r, 0), loy = tile_lo(TS, ty, r, 0);
      const int qx = tile_lo(TS, tx, r + 1, 0), qy = tile_lo(TS, ty, r + 1, 0);
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const double *par = s_v[f] + SH::offset(r + 1) - SH::size(0);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          if (own[i].r != r) continue;
          const int Px = lox + own[i].jx, Py = loy + own[i].jy;
          const int xl = (Px >> 1) - qx, xh = ((Px + 1) >> 1) - qx;
          const int yl = (Py >> 1) - qy, yh = ((Py + 1) >> 1) - qy;
          s_v[f][SH::offset(r) - SH::size(0) + own[i].j] +=
              0.25 * (par[yl * pn + xl] + par[yl * pn + xh] + par[yh * pn + xl] + par[yh * pn + xh]);
        }
      }
    }
    wave_sync();
    // (C) the fields at the lane's nodes (own and ring) into LDS
    double tj[2][3];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      tj[f][0] = s_t[f][0];
      tj[f][1] = s_t[f][1];
      tj[f][2] = s_t[f][2];
    }
    if (n + 1 < n1) take_next();
    wave_sync();
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int e = 0; e <= EF; ++e) {
        if (e == EF && !has_ring) continue;
        const int x = e < EF ? fx : rx, y = e < EF ? fy0 + e : ry;
        double v = tj[f][0] * rc[e][0] + tj[f][1] * rc[e][1] + tj[f][2] * rc[e][2];
        if (R >= 1) v += lev1(s_v[f], x, y);
        if (f == 0) v += basev[e];
        s_f[f][y * NP + x] = v;
      }
    }
    wave_sync();
    // (D) element forms of the lane's four elements: rows fy0 .. fy0+4 of
    // columns fx, fx + 1
    double w[EF + 1][2], u[EF + 1][2];
#pragma unroll
    for (int e = 0; e <= EF; ++e) {
      w[e][0] = s_f[0][(fy0 + e) * NP + fx];
      w[e][1] = s_f[0][(fy0 + e) * NP + fx + 1];
      u[e][0] = s_f[1][(fy0 + e) * NP + fx];
      u[e][1] = s_f[1][(fy0 + e) * NP + fx + 1];
    }
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < EF; ++e) {
      // Q1 element forms with the 1-D mass m = h/6 [2 1; 1 2] and stiffness
      // k = 1/h [1 -1; -1 1]: mass m_y (x) m_x, stiffness c^2 (m_y (x) k_x + k_y (x) m_x)
      const double ul0 = u[e][0], ul1 = u[e][1], uh0 = u[e + 1][0], uh1 = u[e + 1][1];
      const double wl0 = w[e][0], wl1 = w[e][1], wh0 = w[e + 1][0], wh1 = w[e + 1][1];
      const double ml = 2.0 * ul0 * ul0 + 2.0 * ul0 * ul1 + 2.0 * ul1 * ul1;
      const double mh = 2.0 * uh0 * uh0 + 2.0 * uh0 * uh1 + 2.0 * uh1 * uh1;
      const double mc = 2.0 * ul0 * uh0 + ul0 * uh1 + ul1 * uh0 + 2.0 * ul1 * uh1;
      const double mass = hx / 6.0 * hy / 6.0 * (2.0 * ml + 2.0 * mh + 2.0 * mc);
      const double gx0 = wl1 - wl0, gx1 = wh1 - wh0;
      const double gy0 = wh0 - wl0, gy1 = wh1 - wl1;
      const double kx = (hy / 6.0) / hx * (2.0 * gx0 * gx0 + 2.0 * gx0 * gx1 + 2.0 * gx1 * gx1);
      const double ky = (hx / 6.0) / hy * (2.0 * gy0 * gy0 + 2.0 * gy0 * gy1 + 2.0 * gy1 * gy1);
      acc += 0.5 * (mass + c2e[e] * (kx + ky));
    }
    // sum over the wave: every RB instants (and at the chunk's end) lane i
    // adds the 64 lane sums of instant i in lane order, instead of a chain of
    // six cross-lane shuffles per instant
    double *s_r = s_r_w[wave];
    const int slot = (n - n0) % RB;
    s_r[slot * RP + lane] = acc;
    if (slot == RB - 1 || n + 1 == n1) {
      wave_sync();
      if (lane <= slot) {
        const double2 *row = reinterpret_cast<const double2 *>(s_r + lane * RP);
        double sum = 0.0;
#pragma unroll 8
        for (int l = 0; l < 32; ++l) {
          const double2 v = row[l];
          sum += v.x;
          sum += v.y;
        }
        part[(long long)(n - slot + lane) * ntileD + tile] = sum;
      }
      wave_sync();
    }
  }
}

// ------------------------------------------------------- small kernels -----

// Fine-grid mass and stiffness stencils (per-element c^2 on the finest mesh).
//   mode 0: mv = M v,  ku = K u
//   mode 1: mv = M v,  ku = gsum - K u      (adjoint of the lift and u0 term)
template <int D>
__device__ __forceinline__ void fine_stencils_body(int N, const double *__restrict__ ce,
                                                   double hx, double hy,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ u,
                                                   double *__restrict__ mv, double *__restrict__ ku,
                                                   const double *__restrict__ gsum, int mode,
                                                   long long gid) {
  const int n = N - 1;
  const long long nsp = (D == 2) ? (long long)n * n : n;
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

template <int D>
__global__ void k_fine_stencils(int N, const double *__restrict__ ce, double hx,
                                double hy, const double *__restrict__ v,
                                const double *__restrict__ u, double *__restrict__ mv,
                                double *__restrict__ ku, const double *__restrict__ gsum,
                                int mode) {
  fine_stencils_body<D>(N, ce, hx, hy, v, u, mv, ku, gsum, mode, gid64());
}

// ------------------------------------------- launches of many problems ------

// Member of the calling block: the last m with first[m] <= blockIdx.x
// (wave-uniform: scalar loads).
__device__ __forceinline__ int many_member(const ManyLaunch &M) {
  const int b = blockIdx.x;
  int lo = 0, hi = M.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (M.first[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// per-call pointer of slot `slot` for member m (own: the struct's pointer)
template <class T>
__device__ __forceinline__ T *many_ptr(const ManyLaunch &M, int slot, int m, T *own) {
  typedef const double *__attribute__((address_space(4))) const cptr_t;
  return slot < 0 ? own : (T *)((cptr_t *)M.ptr)[(long long)slot * M.nprob + M.prob[m]];
}
// member m's argument struct, read through the scalar cache (the array is
// never written during the launch)
template <class A>
__device__ __forceinline__ const A &many_args(const ManyLaunch &M, int m) {
  typedef const __attribute__((address_space(4))) A cargs_t;
  return *(const A *)((cargs_t *)M.args + m);
}

template <int D, int TS, int TB, int NT, int STENCIL, int NC0>
__global__ void __launch_bounds__(NT, SG_WPE) k_restrict_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;  // padding of the member's block range
  const RestrictArgs &A = many_args<RestrictArgs>(M, m);
  const double *X = many_ptr(M, M.s0, m, A.X);
  if (X == nullptr) return;
  restrict_body<D, TS, TB, NT, STENCIL, NC0>(A, X, lin);
}
template <int STENCIL, int NC0>
__global__ void __launch_bounds__(256, SG_WPEW) k_restrict_w_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const RestrictArgs &A = many_args<RestrictArgs>(M, m);
  const double *X = many_ptr(M, M.s0, m, A.X);
  if (X == nullptr) return;
  restrict_w_body<STENCIL, NC0>(A, X, lin);
}
template <int D, int TS, int TB, int NT, int MODE, int NC0>
__global__ void __launch_bounds__(NT, SG_WPE) k_prolong_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const ProlongArgs &A = many_args<ProlongArgs>(M, m);
  double *out = many_ptr(M, M.s1, m, A.out);
  if (out == nullptr) return;
  prolong_body<D, TS, TB, NT, MODE, NC0>(A, many_ptr(M, M.s0, m, A.base), out, lin);
}
__global__ void __launch_bounds__(256, SG_WPEP) k_prolong_w_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const ProlongArgs &A = many_args<ProlongArgs>(M, m);
  double *out = many_ptr(M, M.s1, m, A.out);
  if (out == nullptr) return;
  prolong_w_body(A, many_ptr(M, M.s0, m, A.base), out, lin);
}
__global__ void __launch_bounds__(256, SG_WPEM) k_prolong_wm_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const ProlongArgs &A = many_args<ProlongArgs>(M, m);
  double *out = many_ptr(M, M.s1, m, A.out);
  if (out == nullptr) return;
  prolong_wm_body(A, many_ptr(M, M.s0, m, A.base), out, lin);
}
template <int D, int TS>
__global__ void __launch_bounds__(256) k_reduce_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const ReduceArgs &A = many_args<ReduceArgs>(M, m);
  const long long b0 = (long long)lin * 256;
  reduce_body<D, TS>(A.g, A.ch, A.in, A.items, A.nitems, A.total, b0 + threadIdx.x,
                     wave_gid0(b0));
}
template <int D>
__global__ void __launch_bounds__(256) k_coarse_restrict_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const ReduceArgs &A = many_args<ReduceArgs>(M, m);
  const long long b0 = (long long)lin * 256;
  coarse_restrict_body<D>(A.g, A.ch, A.in, A.items, A.nitems, A.total,
                          b0 + threadIdx.x, wave_gid0(b0));
}
template <int D>
__global__ void __launch_bounds__(256) k_coarse_pyramid_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const CoarseArgs &A = many_args<CoarseArgs>(M, m);
  coarse_pyramid_body<D>(A.g, A.in, A.out, lin);
}
template <int D>
__global__ void __launch_bounds__(256) k_prolong_coarse_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const CoarseArgs &A = many_args<CoarseArgs>(M, m);
  prolong_coarse_body<D>(A.g, A.ch, A.out, lin);
}
template <int D>
__global__ void __launch_bounds__(256) k_fine_stencils_many(const ManyLaunch M) {
  const int m = many_member(M), lin = blockIdx.x - M.first[m];
  if (lin >= M.nblk[m]) return;
  const StencilArgs &A = many_args<StencilArgs>(M, m);
  double *mv = many_ptr(M, M.s2, m, A.mv);
  double *ku = many_ptr(M, M.s3, m, A.ku);
  fine_stencils_body<D>(A.N, A.ce, A.hx, A.hy, many_ptr(M, M.s0, m, A.v),
                        many_ptr(M, M.s1, m, A.u), mv, ku, A.gsum, A.mode,
                        (long long)lin * 256 + threadIdx.x);
}

// Energy of finest-mesh functions, slab by slab (Sec. 6.3): for slab k,
//   E_k = 1/2 int (ut_k)^2 dx + 1/2 int c^2 |grad w_k|^2 dx
// with ut_k, w_k the P1 (d=1) / Q1 (d=2) functions of the nodal values
// Ut[k], W[k] (zero on the boundary), integrated exactly element by element
// (every element term is a positive semi-definite form, so no cancellation
// between elements).  Grid (nblk, K): in 2-D thread x walks the column of
// elements ex = x from the bottom row up, carrying the values of the row
// below (two new values per field and element, coalesced across the
// threads); in 1-D one element per thread.  Each block sums its threads in
// a fixed tree order into part[k][blk].
template <int D>
__global__ void __launch_bounds__(256) k_energy_part(int N, const double *__restrict__ ce,
                                                     double hx, double hy,
                                                     const double *__restrict__ W,
                                                     const double *__restrict__ Ut,
                                                     double *__restrict__ part) {
  __shared__ double s_red[256];
  const int n = N - 1;
  const long long nsp = (D == 2) ? (long long)n * n : n;
  const int k = blockIdx.y;
  const double *w = W + (long long)k * nsp, *ut = Ut + (long long)k * nsp;
  const int ex = blockIdx.x * blockDim.x + threadIdx.x;  // element (column in 2-D)
  double acc = 0.0;
  if (ex < N) {
    if (D == 1) {
      const double u0 = ex >= 1 ? ut[ex - 1] : 0.0, u1 = ex + 1 <= n ? ut[ex] : 0.0;
      const double w0 = ex >= 1 ? w[ex - 1] : 0.0, w1 = ex + 1 <= n ? w[ex] : 0.0;
      // mass h/6 [2 1; 1 2], stiffness c^2/h [1 -1; -1 1]
      acc = 0.5 * (hx / 6.0 * (2.0 * u0 * u0 + 2.0 * u0 * u1 + 2.0 * u1 * u1) +
                   ce[ex] / hx * (w1 - w0) * (w1 - w0));
    } else {
      // node columns ex and ex + 1; node rows 0 and N are on the boundary
      const bool c0 = ex >= 1, c1 = ex + 1 <= n;
      const int x0 = c0 ? ex - 1 : 0, x1 = c1 ? ex : 0;
      double ul0 = 0.0, ul1 = 0.0, wl0 = 0.0, wl1 = 0.0;  // row below (node row 0)
      for (int ey = 0; ey < N; ++ey) {
        double uh0 = 0.0, uh1 = 0.0, wh0 = 0.0, wh1 = 0.0;  // node row ey + 1
        if (ey + 1 <= n) {
          const long long r = (long long)ey * n;
          uh0 = c0 ? ut[r + x0] : 0.0;
          uh1 = c1 ? ut[r + x1] : 0.0;
          wh0 = c0 ? w[r + x0] : 0.0;
          wh1 = c1 ? w[r + x1] : 0.0;
        }
        // Q1 element forms with the 1-D mass m = h/6 [2 1; 1 2] and stiffness
        // k = 1/h [1 -1; -1 1]: mass m_y (x) m_x, stiffness c^2 (m_y (x) k_x + k_y (x) m_x)
        const double ml = 2.0 * ul0 * ul0 + 2.0 * ul0 * ul1 + 2.0 * ul1 * ul1;
        const double mh = 2.0 * uh0 * uh0 + 2.0 * uh0 * uh1 + 2.0 * uh1 * uh1;
        const double mc = 2.0 * ul0 * uh0 + ul0 * uh1 + ul1 * uh0 + 2.0 * ul1 * uh1;
        const double mass = hx / 6.0 * hy / 6.0 * (2.0 * ml + 2.0 * mh + 2.0 * mc);
        const double gx0 = wl1 - wl0, gx1 = wh1 - wh0;  // x differences of the two rows
        const double gy0 = wh0 - wl0, gy1 = wh1 - wl1;  // y differences of the two columns
        const double kx = (hy / 6.0) / hx * (2.0 * gx0 * gx0 + 2.0 * gx0 * gx1 + 2.0 * gx1 * gx1);
        const double ky = (hx / 6.0) / hy * (2.0 * gy0 * gy0 + 2.0 * gy0 * gy1 + 2.0 * gy1 * gy1);
        acc += 0.5 * (mass + ce[(long long)ey * N + ex] * (kx + ky));
        ul0 = uh0; ul1 = uh1; wl0 = wh0; wl1 = wh1;
      }
    }
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) s_red[threadIdx.x] += s_red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)k * gridDim.x + blockIdx.x] = s_red[0];
}

// E[k] = sum_b part[k][b]: one wave per instant, lane l adding the partials
// b = l, l + 64, ..., then a butterfly (a fixed order)
__global__ void __launch_bounds__(64) k_energy_sum(int K, int nblk,
                                                   const double *__restrict__ part,
                                                   double *__restrict__ E) {
  const int k = blockIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += part[(long long)k * nblk + b];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) E[k] = s;
}


// L^2(Q_T) error by quadrature: W[k] holds u_h at the k-th Gauss instant on
// the finest nodes, UQ[k] the exact solution at the 2 x 2 (2-D) or 2 (1-D)
// Gauss points of every finest element (point 2 e + g of axis-element e,
// g = 0 at (1 - 1/sqrt 3) h / 2, g = 1 at (1 + 1/sqrt 3) h / 2 from the
// element's left end).  One thread per element (a column of elements in 2-D,
// walked bottom to top); per instant and block the sums of w (u - u_h)^2 and
// w u^2 over the block's elements and points, w the spatial Gauss weight.
template <int D>
__global__ void __launch_bounds__(256) k_l2_part(int N, double hx, double hy,
                                                 const double *__restrict__ W,
                                                 const double *__restrict__ UQ,
                                                 double *__restrict__ part) {
  __shared__ double s_e[256], s_n[256];
  const int n = N - 1;
  const long long nsp = (D == 2) ? (long long)n * n : n;
  const long long nq = (D == 2) ? 4LL * N * N : 2LL * N;
  const int k = blockIdx.y;
  const double *w = W + (long long)k * nsp, *uq = UQ + (long long)k * nq;
  const int ex = blockIdx.x * blockDim.x + threadIdx.x;
  const double g0 = 0.5 - 0.5 / sqrt(3.0), g1 = 0.5 + 0.5 / sqrt(3.0);  // local points
  const double xi[2] = {g0, g1};
  double ae = 0.0, an = 0.0;
  if (ex < N) {
    const bool c0 = ex >= 1, c1 = ex + 1 <= n;
    const int x0 = c0 ? ex - 1 : 0, x1 = c1 ? ex : 0;
    if (D == 1) {
      const double w0 = c0 ? w[x0] : 0.0, w1 = c1 ? w[x1] : 0.0;
      const double wt = 0.5 * hx;
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const double uh = (1.0 - xi[g]) * w0 + xi[g] * w1, u = uq[2 * ex + g];
        ae += wt * (u - uh) * (u - uh);
        an += wt * u * u;
      }
    } else {
      const double wt = 0.25 * hx * hy;
      double wl0 = 0.0, wl1 = 0.0;  // node row ey (row 0 is on the boundary)
      for (int ey = 0; ey < N; ++ey) {
        double wh0 = 0.0, wh1 = 0.0;  // node row ey + 1
        if (ey + 1 <= n) {
          const long long r = (long long)ey * n;
          wh0 = c0 ? w[r + x0] : 0.0;
          wh1 = c1 ? w[r + x1] : 0.0;
        }
#pragma unroll
        for (int gy = 0; gy < 2; ++gy) {
          const double *uqr = uq + (long long)(2 * ey + gy) * (2 * N) + 2 * ex;
#pragma unroll
          for (int gx = 0; gx < 2; ++gx) {
            const double lo = (1.0 - xi[gx]) * wl0 + xi[gx] * wl1;
            const double hi = (1.0 - xi[gx]) * wh0 + xi[gx] * wh1;
            const double uh = (1.0 - xi[gy]) * lo + xi[gy] * hi, u = uqr[gx];
            ae += wt * (u - uh) * (u - uh);
            an += wt * u * u;
          }
        }
        wl0 = wh0;
        wl1 = wh1;
      }
    }
  }
  s_e[threadIdx.x] = ae;
  s_n[threadIdx.x] = an;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) {
      s_e[threadIdx.x] += s_e[threadIdx.x + h];
      s_n[threadIdx.x] += s_n[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((long long)k * gridDim.x + blockIdx.x) * 2] = s_e[0];
    part[((long long)k * gridDim.x + blockIdx.x) * 2 + 1] = s_n[0];
  }
}

// out[0] = sum_k wt[k] sum_b part[k][b][0], out[1] likewise with [1]: one
// wave, lane l taking the instants l, l + 64, ..., then a butterfly
__global__ void __launch_bounds__(64) k_l2_sum(int K, int nblk, const double *__restrict__ part,
                                               const double *__restrict__ wt,
                                               double *__restrict__ out) {
  double se = 0.0, sn = 0.0;
  for (int k = threadIdx.x; k < K; k += 64) {
    double e = 0.0, m = 0.0;
    for (int b = 0; b < nblk; ++b) {
      e += part[((long long)k * nblk + b) * 2];
      m += part[((long long)k * nblk + b) * 2 + 1];
    }
    se += wt[k] * e;
    sn += wt[k] * m;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    se += __shfl_xor(se, o, 64);
    sn += __shfl_xor(sn, o, 64);
  }
  if (threadIdx.x == 0) {
    out[0] = se;
    out[1] = sn;
  }
}

// b_c[i][K] = sum_q D_b[i][q] Z_c[q][K] + psi_i'(0) MV_a[K] - g_b[i] KU_a[K]
__global__ void k_post_load(const CompDesc *__restrict__ cd, int ncomp, long long total) {
  const long long gid = gid64();
  const int ci = find_item(cd, ncomp, gid, wave_gid0((long long)blockIdx.x * blockDim.x));
  if (gid >= total) return;
  const CompDesc &C = cref(cd, ci);
  const long long loc = gid - C.start;
  const int i = (int)loc / C.nsp;  // a component holds fewer than 2^31 values
  const int K = (int)loc - i * C.nsp;
  const double *Z = C.z;
  const KernelTables *kt = &cref(C.kt, 0);
  double v = gld(kt->Dlo[C.b], i) * Z[loc];
  if (i + 1 < C.nq) v += gld(kt->Dhi[C.b], i) * Z[loc + C.nsp];
  if (i == 0 && C.mv != nullptr) v += gld(kt->Dlo[C.b], 0) * gld(C.mv, K);
  if (C.ku != nullptr) v -= gld(kt->g[C.b], i) * gld(C.ku, K);
  gst(C.data, loc, v);
}

// zeta_c[q][K] = sum_i D_b[i][q] z_c[i][K]   (transpose of the above)
__global__ void k_post_adjoint(const CompDesc *__restrict__ cd, int ncomp,
                               long long total) {
  const long long gid = gid64();
  const int ci = find_item(cd, ncomp, gid, wave_gid0((long long)blockIdx.x * blockDim.x));
  if (gid >= total) return;
  const CompDesc &C = cref(cd, ci);
  const long long loc = gid - C.start;
  const int q = (int)loc / C.nsp;  // a component holds fewer than 2^31 values
  const KernelTables *kt = &cref(C.kt, 0);
  const double *Z = C.z;
  double v = gld(kt->Dlo[C.b], q) * Z[loc];
  if (q >= 1) v += gld(kt->Dhi[C.b], q - 1) * Z[loc - C.nsp];
  gst(C.data, loc, v);
}

// fv_a[K] = sum_c psi_0'(0) z_c[0][K];  fu_a[K] = sum_c sum_i g_b[i] z_c[i][K].
// Levels whose components have long time levels use one wave per node (lanes
// split the time sum, then a shuffle reduction); the others one thread.
__global__ void k_adjoint_fields(const LevelDesc *__restrict__ ld, int nlev,
                                 long long total) {
  const long long gid = gid64();
  const int l = find_item(ld, nlev, gid, wave_gid0((long long)blockIdx.x * blockDim.x));
  if (gid >= total) return;
  const LevelDesc &L = cref(ld, l);
  const CompDesc *cd = L.cd;
  const KernelTables *kt = &cref(L.kt, 0);
  const long long rel = gid - L.start;
  const int lane = L.wave ? (int)(rel & 63) : 0, step = L.wave ? 64 : 1;
  const long long K = L.wave ? rel >> 6 : rel;
  if (K >= L.nsp) return;  // whole waves in wave levels
  double fv = 0.0, fu = 0.0;
  for (int t = 0; t < 2; ++t) {
    const int c = t == 0 ? L.c0 : L.c1;
    if (c < 0) continue;
    const CompDesc &C = cref(cd, c);
    const double *Z = C.z;
    if (lane == 0) fv += gld(kt->Dlo[C.b], 0) * Z[K];
    const gptr<const double> gb = to_g(kt->g[C.b]);
    for (int i = lane; i < C.nq; i += step) fu += gb[i] * Z[(long long)i * C.nsp + K];
  }
  if (L.wave) {
#pragma unroll
    for (int dlt = 32; dlt >= 1; dlt >>= 1) fu += __shfl_xor(fu, dlt);
    if (lane != 0) return;
  }
  gst(L.fv, K, fv);
  gst(L.fu, K, fu);
}

// Batched C = A B (row major) on the FP64 matrix cores.  Block tiles of
// kGemmTile square, each wave a 32x32 sub-tile of 2x2 v_mfma_f64_16x16x4
// blocks; K in
// steps of SG_GEMM_BK through LDS, the next K tile prefetched in registers.
// Operand layout of the 16x16x4 instruction (lane l of the wave):
//   a = A[l % 16][l / 16],  b = B[l / 16][l % 16],
//   result element r of the lane = D[l / 16 + 4 r][l % 16].
typedef double sg_double4 __attribute__((ext_vector_type(4)));

// FOLD = 1 / 2: descriptors with nref > 0 fold the summed index k of A's
// columns / B's rows with its reflection nref-1-k, and their results are the
// outputs of one parity, stored at every other column / row of C.
// FOLD = 3 / 4: plain products whose A / B operand is read transposed (every
// descriptor of the list has ta / tb set); FOLD = 0: plain products.
#ifndef SG_GEMM_BK
#define SG_GEMM_BK 64
#endif
template <int FOLD>
__global__ void __launch_bounds__(kGemmThreads) k_gemm(const GemmDesc *__restrict__ descs,
                                                      int ndesc) {
  // K steps of SG_GEMM_BK: with 64 each step is 64 MFMAs per wave (about
  // 1.7 us of matrix work), enough to cover the global-load latency of the
  // next step's operands, which are prefetched into registers meanwhile
  constexpr int NT = kGemmThreads, W = SG_GEMM_W;
  constexpr int BM = kGemmTile, BN = kGemmTile, BK = SG_GEMM_BK;
  constexpr int EA = BM * BK / NT, EB = BK * BN / NT;  // staged values per thread
  __shared__ double As[BM][BK + 1];
  __shared__ double Bs[BK][BN + 2];
  // this tile's descriptor: the last one whose first tile is <= blockIdx.x
  // (tile0 ascends); one gather of tile0 per lane for 64 descriptors at a
  // time instead of a chain of dependent scalar loads
  int di = 0;
  for (int base = 0; base < ndesc; base += 64) {
    const int i = base + (int)(threadIdx.x & 63);
    const unsigned long long le = __ballot(i < ndesc && descs[i].tile0 <= (int)blockIdx.x);
    di += __popcll(le);
    if (le != ~0ull) break;
  }
  di = __builtin_amdgcn_readfirstlane(di - 1);
  const GemmDesc &Dd = cref(descs, di);
  int t = blockIdx.x - Dd.tile0;
  const int per = Dd.tm * Dd.tn;
  const int bidx = t / per;
  t -= bidx * per;
  const int tmi = t / Dd.tn, tni = t - tmi * Dd.tn;
  const double *Ap = Dd.A + bidx * Dd.sA;
  const double *Bp = Dd.B + bidx * Dd.sB;
  double *Cp = Dd.C + bidx * Dd.sC;
  const int row0 = tmi * BM, col0 = tni * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / W) * 32, wn = (wave % W) * 32;
  const int M = Dd.M, N = Dd.N, K = Dd.K;
  // folding: k < h pairs with its reflection, k = h (even parity only) is
  // the unpaired middle index
  const bool fd = FOLD != 0 && Dd.nref > 0;
  const int nr1 = Dd.nref - 1, hmid = nr1 / 2;
  const double sgn = Dd.par ? -1.0 : 1.0;
  // global -> register staging; loads go to clamped valid addresses and are
  // selected, not branched
  // staged element e of this thread: (m, k) of the A tile, (kb, n) of the B
  // tile; consecutive threads take consecutive addresses of the stored
  // operand (along k for A, n for B, or along m / kb when transposed)
  constexpr bool ta = FOLD == 3, tb = FOLD == 4;
  auto a_at = [&](int e, int &m, int &k) {
    const int i = tid + e * NT;
    if (ta) { m = i % BM; k = i / BM; } else { m = i / BK; k = i % BK; }
  };
  auto b_at = [&](int e, int &kb, int &n) {
    const int i = tid + e * NT;
    if (tb) { kb = i % BK; n = i / BK; } else { kb = i / BN; n = i % BN; }
  };
  // Offsets inside one descriptor's operands are 32-bit (checked on the host).
  // The reflected partner of a folded operand is loaded unconditionally (from
  // a valid address when it is not used) and added with weight sgn, or 0 at
  // the unpaired middle index: a conditional add lets the compiler move the
  // load into a branch that waits for it at once, which serialises the
  // tile's loads (one memory latency per element instead of one per tile).
  const int lda = Dd.lda, ldb = Dd.ldb;
  double ra[EA], rb[EB];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int m, k;
      a_at(e, m, k);                                // A: BM x BK
      const int gm = row0 + m, gk = k0 + k;
      const bool oka = gm < M && gk < K;
      const int ia = oka ? (ta ? gk * lda + gm : gm * lda + gk) : 0;
      double va = Ap[ia];
      if (FOLD == 1) {
        const double vr = Ap[fd && oka ? ia + nr1 - 2 * gk : 0];
        va = fma(fd && gk != hmid ? sgn : 0.0, vr, va);
      }
      ra[e] = oka ? va : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int kb, n;
      b_at(e, kb, n);                               // B: BK x BN
      const int gkb = k0 + kb, gn = col0 + n;
      const bool okb = gkb < K && gn < N;
      const int ib = okb ? (tb ? gn * ldb + gkb : gkb * ldb + gn) : 0;
      double vb = Bp[ib];
      if (FOLD == 2) {
        const double vr = Bp[fd && okb ? (nr1 - gkb) * ldb + gn : 0];
        vb = fma(fd && gkb != hmid ? sgn : 0.0, vr, vb);
      }
      rb[e] = okb ? vb : 0.0;
    }
  };
  sg_double4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = sg_double4{0.0, 0.0, 0.0, 0.0};
  load_tile(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int m, k;
      a_at(e, m, k);
      As[m][k] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int kb, n;
      b_at(e, kb, n);
      Bs[kb][n] = rb[e];
    }
    __syncthreads();
    if (k0 + BK < K) load_tile(k0 + BK);
    const int kend = min(BK, K - k0);  // the rest of the tile is zero
    for (int kk = 0; kk < kend; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = row0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int gn = col0 + wn + j * 16 + (lane & 15);
        const int cm = FOLD == 2 && fd ? 2 * gm + Dd.par : gm;
        const int cn = FOLD == 1 && fd ? 2 * gn + Dd.par : gn;
        if (gm < M && gn < N) Cp[(long long)cm * Dd.ldc + cn] = acc[i][j][r];
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
// (x.h + x.l) * (y.h + y.l) to double-double accuracy
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
#pragma clang fp contract(off)
  dd p = two_prod(x.h, y.h);
  p.l += x.h * y.l + x.l * y.h;
  return two_sum(p.h, p.l);
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
  if (d == 1 || S.flat) {
    m = gld(mt->mx[a], j);
    kap = S.c2 * gld(mt->kx[a], j);
  } else {
    const int jx = j % na, jy = j / na;
    const double mx = gld(mt->mx[a], jx), kx = gld(mt->kx[a], jx);
    const double my = gld(mt->my[a], jy), ky = gld(mt->ky[a], jy);
    m = my * mx;
    kap = S.c2 * (ky * mx + my * kx);
  }
}

__global__ void __launch_bounds__(64) k_time_factor(const SolveDesc *__restrict__ sds,
                                                    int nsd, long long total) {
  const long long wbase = (long long)blockIdx.x * 64;
  const SolveDesc &S = cref(sds, find_solve(sds, nsd, wbase));
  const KernelTables *kt = &cref(S.kt, 0);
  const ModeTables *mt = &cref(S.mt, 0);
  const int d = S.d;
  const long long gid = wbase + threadIdx.x;
  const int j = (int)(gid - S.thread0);
  if (gid >= total || j >= S.nmodes) return;
  const int b = S.b, nq = S.nq, nm = S.nmodes;
  double m, kap;
  mode_scalars(S, j, mt, d, m, kap);
  const gptr<const double> Ab = to_g(kt->A[b]), Bb = to_g(kt->B[b]);
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

// Inclusive scan across the wave, in recurrence order, of the affine maps
// S -> c + H S (S = (v_prev, v_prev2)) of the lanes' row blocks; (s1, s2) is
// the state entering this lane's block (zero for the first block).
__device__ __forceinline__ void wave_scan_maps(bool fwd, int lane, double c1, double c2,
                                               double h11, double h12, double h21, double h22,
                                               double &s1, double &s2) {
#pragma unroll
  for (int dlt = 1; dlt < 64; dlt <<= 1) {
    const int src = fwd ? lane - dlt : lane + dlt;
    const int sl = src < 0 ? 0 : (src > 63 ? 63 : src);
    const double pc1 = __shfl(c1, sl), pc2 = __shfl(c2, sl);
    const double p11 = __shfl(h11, sl), p12 = __shfl(h12, sl);
    const double p21 = __shfl(h21, sl), p22 = __shfl(h22, sl);
    if (src >= 0 && src <= 63) {
      // mine o theirs: S -> c + H (pc + P S)
      const double nc1 = c1 + h11 * pc1 + h12 * pc2;
      const double nc2 = c2 + h21 * pc1 + h22 * pc2;
      const double n11 = h11 * p11 + h12 * p21, n12 = h11 * p12 + h12 * p22;
      const double n21 = h21 * p11 + h22 * p21, n22 = h21 * p12 + h22 * p22;
      c1 = nc1; c2 = nc2; h11 = n11; h12 = n12; h21 = n21; h22 = n22;
    }
  }
  const int prev = fwd ? lane - 1 : lane + 1;
  const int psl = prev < 0 ? 0 : (prev > 63 ? 63 : prev);
  s1 = __shfl(c1, psl);
  s2 = __shfl(c2, psl);
  if (prev < 0 || prev > 63) s1 = s2 = 0.0;
}

__device__ __forceinline__ double wave_fmax(double v) {
#pragma unroll
  for (int dlt = 32; dlt >= 1; dlt >>= 1) v = fmax(v, __shfl_xor(v, dlt));
  return v;
}

// One mode of a time level of nq <= 64 BK rows (BK = 1 or 2; more rows per
// lane raise the kernel's register count past two waves per SIMD) on one
// wave with every row in registers: lane l holds rows l BK .. l BK + BK - 1 (the block layout of the
// general one-wave path for the same nq).  The sweeps, the scans and the
// double-double refinement are those of the general path, in the same order,
// but no pass makes a memory round trip: the residual's rows beyond the
// lane's block come from the lanes beside.  Row indices are constants (a
// register array indexed at run time would be placed in scratch memory).
template <int BK, bool TR>
__device__ __forceinline__ void wave_solve_regs(int lane, int nq, int refine, long long nm, int j,
                                                double m, double kap, gptr<const double> Ab,
                                                gptr<const double> Bb, gptr<const double> Al,
                                                gptr<const double> Bl, const double *L1,
                                                const double *L2, const double *UD,
                                                const double *U1, const double *U2,
                                                double *rhs) {
  auto idx = [&](int i) -> long long { return (long long)i * nm + j; };
  const int r0 = min(lane * BK, nq), cnt = min(r0 + BK, nq) - r0;
  // row t of the lane: coefficients of the forward-in-time sweep (P = 0: L,
  // or U^T) and of the backward one (P = 1: U, or L^T); the solution x, the
  // right-hand side b, the intermediate y
  double pa[2][BK], pb1[2][BK], pb2[2][BK], x[BK], b[BK], y[BK];
#pragma unroll
  for (int t = 0; t < BK; ++t) {
    pa[0][t] = pb1[0][t] = pb2[0][t] = pa[1][t] = pb1[1][t] = pb2[1][t] = 0.0;
    x[t] = b[t] = y[t] = 0.0;
    if (t < cnt) {
      const int i = r0 + t;
      b[t] = rhs[idx(i)];
      if (!TR) {
        pa[0][t] = 1.0; pb1[0][t] = L1[idx(i)]; pb2[0][t] = L2[idx(i)];
        pa[1][t] = UD[idx(i)]; pb1[1][t] = U1[idx(i)]; pb2[1][t] = U2[idx(i)];
      } else {
        pa[0][t] = UD[idx(i)];
        pb1[0][t] = i >= 1 ? U1[idx(i - 1)] : 0.0;
        pb2[0][t] = i >= 2 ? U2[idx(i - 2)] : 0.0;
        pa[1][t] = 1.0;
        pb1[1][t] = i + 1 < nq ? L1[idx(i + 1)] : 0.0;
        pb2[1][t] = i + 2 < nq ? L2[idx(i + 2)] : 0.0;
      }
    }
  }
  auto spass = [&](int P, const double (&in)[BK], double (&out)[BK],
                   bool add) __attribute__((always_inline)) -> double {
    const bool fwd = P == 0;
    double c1 = 0.0, c2 = 0.0, h11 = 1.0, h21 = 0.0, h12 = 0.0, h22 = 1.0;
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      const int t = fwd ? k : BK - 1 - k;
      if (t >= cnt) continue;
      const double a = pa[P][t], b1 = pb1[P][t], b2 = pb2[P][t];
      const double v = a * (in[t] - b1 * c1 - b2 * c2);
      c2 = c1; c1 = v;
      const double g1 = -a * (b1 * h11 + b2 * h21);
      h21 = h11; h11 = g1;
      const double g2 = -a * (b1 * h12 + b2 * h22);
      h22 = h12; h12 = g2;
    }
    double s1, s2;
    wave_scan_maps(fwd, lane, c1, c2, h11, h12, h21, h22, s1, s2);
    double xm = 0.0;
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      const int t = fwd ? k : BK - 1 - k;
      if (t >= cnt) continue;
      const double v = pa[P][t] * (in[t] - pb1[P][t] * s1 - pb2[P][t] * s2);
      s2 = s1; s1 = v;
      out[t] = add ? out[t] + v : v;
      xm = fmax(xm, fabs(v));
    }
    return xm;
  };
  auto apply = [&](const double (&R)[BK], bool add) __attribute__((always_inline)) -> double {
    spass(0, R, y, false);
    return wave_fmax(spass(1, y, x, add));
  };
  apply(b, false);
  for (int it = 0; it < refine; ++it) {
    // rows just outside the block: the two before and the two after it
    // (lanes two and one to each side when BK = 1, else the lanes beside)
    const int sm1 = lane > 0 ? lane - 1 : 0, sp1 = lane < 63 ? lane + 1 : 63;
    const int sm2 = lane > 1 ? lane - 2 : 0, sp2 = lane < 62 ? lane + 2 : 63;
    const double xm1 = __shfl(x[BK - 1], sm1);
    const double xm2 = BK >= 2 ? __shfl(x[BK >= 2 ? BK - 2 : 0], sm1) : __shfl(x[0], sm2);
    const double xp1 = __shfl(x[0], sp1);
    const double xp2 = BK >= 2 ? __shfl(x[BK >= 2 ? 1 : 0], sp1) : __shfl(x[0], sp2);
    // x at block position u = -2 .. BK + 1
    auto xat = [&](int u) __attribute__((always_inline)) -> double {
      return u == -2 ? xm2 : u == -1 ? xm1 : u == BK ? xp1 : u == BK + 1 ? xp2 : x[u < 0 ? 0 : (u >= BK ? BK - 1 : u)];
    };
    double xmax = 0.0, res[BK];
#pragma unroll
    for (int t = 0; t < BK; ++t) {
      res[t] = 0.0;
      if (t >= cnt) continue;
      {
        // residual row i: b_i - (op(E) x)_i, in double-double, as resid_row
#pragma clang fp contract(off)
        const int i = r0 + t;
        dd acc = {b[t], 0.0};
#pragma unroll
        for (int off = -2; off <= 2; ++off) {
          const int jj = i + off;
          if (jj < 0 || jj >= nq) continue;
          const int r = TR ? jj : i, c = TR ? 2 - off : off + 2;
          const double xv = xat(t + off);
          if (off == 0) xmax = fmax(xmax, fabs(xv));
          dd t1 = triple(m, Ab[r * 5 + c], xv);
          dd t2 = triple(kap, Bb[r * 5 + c], xv);
          t1.l = fma(m * Al[r * 5 + c], xv, t1.l);
          t2.l = fma(kap * Bl[r * 5 + c], xv, t2.l);
          acc = dd_add(acc, {-t1.h, -t1.l});
          acc = dd_add(acc, {-t2.h, -t2.l});
        }
        res[t] = acc.h + acc.l;
      }
    }
    xmax = wave_fmax(xmax);
    const double dmax = apply(res, true);
    if (dmax <= 1e-15 * xmax) break;
  }
#pragma unroll
  for (int t = 0; t < BK; ++t)
    if (t < cnt) rhs[idx(r0 + t)] = x[t];
}

// TR: the transposed (adjoint) systems; one instantiation per direction
// keeps each kernel's code to the path it runs
template <int TR>
__global__ void __launch_bounds__(64) k_time_solve(const SolveDesc *__restrict__ sds,
                                                   int nsd, long long total) {
  // rows per register chunk of a substitution / of the residual (thread path)
#ifndef SG_CH
#define SG_CH 8
#endif
#ifndef SG_CR
#define SG_CR 8
#endif
#ifndef SG_CW
#define SG_CW 4
#endif
  constexpr int CH = SG_CH;
  constexpr int CR = SG_CR;
  constexpr int CW = SG_CW;  // rows per chunk of a lane's block (wave path)
  const long long wbase = (long long)blockIdx.x * 64;
  const SolveDesc &S = cref(sds, find_solve(sds, nsd, wbase));
  const KernelTables *kt = &cref(S.kt, 0);
  const ModeTables *mt = &cref(S.mt, 0);
  const int d = S.d;
  const int lane = threadIdx.x;
  const bool wave = S.wave != 0;
  // wave path: one mode per wave; thread path: one mode per thread
  const int j = wave ? (int)((wbase - S.thread0) >> 6) : (int)(wbase + lane - S.thread0);
  if (wbase + lane >= total || j >= S.nmodes) return;  // uniform in the wave path
  const int b = S.b, nq = S.nq, nm = S.nmodes;
  double m, kap;
  mode_scalars(S, j, mt, d, m, kap);
  const gptr<const double> Ab = to_g(kt->A[b]), Bb = to_g(kt->B[b]), Al = to_g(kt->Alo[b]),
                          Bl = to_g(kt->Blo[b]);
  constexpr bool tr = TR != 0;
  double *rhs = S.rhs;
  const long long plane = (long long)nq * nm;
  const double *L1 = S.fac, *L2 = L1 + plane, *UD = L2 + plane, *U1 = UD + plane,
               *U2 = U1 + plane;
  double *Y = S.scratch, *B0 = Y + plane;
  auto idx = [&](int i) -> long long { return (long long)i * nm + j; };

  // residual row i: b_i - (op(E) x)_i with E from the double-double time
  // matrices, accumulated in double-double; also folds |x_i| into xmax
  auto resid_row = [&](int i, double &xmax) -> double {
#pragma clang fp contract(off)
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
    return acc.h + acc.l;
  };

  if (wave) {
    // ---- wave-parallel path: lane l owns rows [l*bk, (l+1)*bk) ----------
    // Each of the four banded triangular recurrences
    //   v_i = a_i (r_i - b1_i v_prev - b2_i v_prev2)
    // is solved block-wise: every lane first derives the affine map of its
    // block on the carried state (v_prev, v_prev2), an inclusive scan of
    // these maps across the wave (in recurrence order) gives every block
    // its entry state, and the block is then swept once more.
    const int bk = (nq + 63) / 64;
    const int r0 = min(lane * bk, nq), r1 = min(r0 + bk, nq);
    auto wave_scan = [&](bool fwd, double c1, double c2, double h11, double h12, double h21,
                         double h22, double &s1, double &s2) __attribute__((always_inline)) {
      wave_scan_maps(fwd, lane, c1, c2, h11, h12, h21, h22, s1, s2);
    };
    auto wave_max = [&](double v) -> double { return wave_fmax(v); };
    auto coefs = [&](int which, int i, const double *Rin, double &a, double &b1, double &b2,
                     double &r) __attribute__((always_inline)) {
      if (which == 0) {
        a = 1.0; b1 = L1[idx(i)]; b2 = L2[idx(i)]; r = Rin[idx(i)];
      } else if (which == 1) {
        a = UD[idx(i)]; b1 = U1[idx(i)]; b2 = U2[idx(i)]; r = Rin[idx(i)];
      } else if (which == 2) {
        a = UD[idx(i)];
        b1 = i >= 1 ? U1[idx(i - 1)] : 0.0;
        b2 = i >= 2 ? U2[idx(i - 2)] : 0.0;
        r = Rin[idx(i)];
      } else {
        a = 1.0;
        b1 = i + 1 < nq ? L1[idx(i + 1)] : 0.0;
        b2 = i + 2 < nq ? L2[idx(i + 2)] : 0.0;
        r = Rin[idx(i)];
      }
    };
    // time levels of up to 128 nodes (at most 2 rows per lane): every row in
    // registers
#define SG_WAVE_REGS(BKV)                                                                   \
  if (bk == BKV) {                                                                          \
    wave_solve_regs<BKV, TR != 0>(lane, nq, S.refine, nm, j, m, kap, Ab, Bb, Al, Bl, L1, L2, \
                                  UD, U1, U2, rhs);                                        \
    return;                                                                                 \
  }
    SG_WAVE_REGS(1)
    SG_WAVE_REGS(2)
#undef SG_WAVE_REGS
    // the lane's rows are visited in chunks of CW whose coefficients are
    // loaded together: one memory latency per chunk instead of one per row
    // on the recurrence's critical path
    auto pass = [&](int which, const double *Rin, double *out,
                    bool add) __attribute__((always_inline)) -> double {
      const bool fwd = (which == 0 || which == 2);
      const int cnt = r1 - r0;
      // step 1: block map  S_out = c + H S_in,  S = (v_prev, v_prev2)
      double c1 = 0.0, c2 = 0.0, h11 = 1.0, h21 = 0.0, h12 = 0.0, h22 = 1.0;
      for (int t0 = 0; t0 < cnt; t0 += CW) {
        double ca[CW], cb1[CW], cb2[CW], cr[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k)
          if (t0 + k < cnt)
            coefs(which, fwd ? r0 + t0 + k : r1 - 1 - t0 - k, Rin, ca[k], cb1[k], cb2[k], cr[k]);
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          if (t0 + k >= cnt) break;
          const double a = ca[k], b1 = cb1[k], b2 = cb2[k];
          const double v = a * (cr[k] - b1 * c1 - b2 * c2);
          c2 = c1; c1 = v;
          const double g1 = -a * (b1 * h11 + b2 * h21);
          h21 = h11; h11 = g1;
          const double g2 = -a * (b1 * h12 + b2 * h22);
          h22 = h12; h12 = g2;
        }
      }
      // step 2: inclusive scan of the maps in recurrence order
      double s1, s2;
      wave_scan(fwd, c1, c2, h11, h12, h21, h22, s1, s2);
      // step 3: sweep the block from its entry state (a chunk's rows are
      // read before any of them is written: out may be Rin)
      double xm = 0.0;
      for (int t0 = 0; t0 < cnt; t0 += CW) {
        double ca[CW], cb1[CW], cb2[CW], cr[CW], old[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k)
          if (t0 + k < cnt) {
            const int i = fwd ? r0 + t0 + k : r1 - 1 - t0 - k;
            coefs(which, i, Rin, ca[k], cb1[k], cb2[k], cr[k]);
            old[k] = add ? out[idx(i)] : 0.0;
          }
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          if (t0 + k >= cnt) break;
          const int i = fwd ? r0 + t0 + k : r1 - 1 - t0 - k;
          const double v = ca[k] * (cr[k] - cb1[k] * s1 - cb2[k] * s2);
          s2 = s1; s1 = v;
          out[idx(i)] = add ? old[k] + v : v;
          xm = fmax(xm, fabs(v));
        }
      }
      __syncthreads();  // rows of other lanes are read by the next sweep
      return xm;
    };
    auto apply = [&](const double *R, bool add) -> double {
      if (!tr) {
        pass(0, R, Y, false);
        return wave_max(pass(1, Y, rhs, add));
      }
      pass(2, R, Y, false);
      return wave_max(pass(3, Y, rhs, add));
    };
    if (S.refine) {
      for (int i0 = r0; i0 < r1; i0 += CW) {
        double v[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k)
          if (i0 + k < r1) v[k] = rhs[idx(i0 + k)];
#pragma unroll
        for (int k = 0; k < CW; ++k)
          if (i0 + k < r1) B0[idx(i0 + k)] = v[k];
      }
      __syncthreads();
    }
    apply(rhs, false);
    for (int it = 0; it < S.refine; ++it) {
      double xmax = 0.0;
      for (int i0 = r0; i0 < r1; i0 += CR) {
        double res[CR];
#pragma unroll
        for (int k = 0; k < CR; ++k)
          if (i0 + k < r1) res[k] = resid_row(i0 + k, xmax);
#pragma unroll
        for (int k = 0; k < CR; ++k)
          if (i0 + k < r1) Y[idx(i0 + k)] = res[k];
      }
      __syncthreads();
      xmax = wave_max(xmax);
      const double dmax = apply(Y, true);
      if (dmax <= 1e-15 * xmax) break;
    }
    return;
  }

  // ---- thread path: one mode per thread, rows in register chunks ---------
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
  if (S.refine) {
    for (int i0 = 0; i0 < nq; i0 += CH) {
      double v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (i0 + k < nq) v[k] = rhs[idx(i0 + k)];
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (i0 + k < nq) B0[idx(i0 + k)] = v[k];
    }
  }
  apply_inverse(rhs, false);
  // refinement: x += op(E)^{-1} (b - op(E) x); stop once the correction is
  // below 1e-15 of the solution (the next one would be below the rounding
  // of x itself)
  for (int it = 0; it < S.refine; ++it) {
    double xmax = 0.0;
    for (int i0 = 0; i0 < nq; i0 += CR) {
      double res[CR];
#pragma unroll
      for (int k = 0; k < CR; ++k)
        if (i0 + k < nq) res[k] = resid_row(i0 + k, xmax);
#pragma unroll
      for (int k = 0; k < CR; ++k)
        if (i0 + k < nq) Y[idx(i0 + k)] = res[k];
    }
    const double dmax = apply_inverse(Y, true);
    if (dmax <= 1e-15 * xmax) break;
  }
}

// ---- block LU solve with double-double refinement (1-D, variable c) -----

// One wave per component.  x <- op(S)^{-1} r with the block LU S = L U in
// space-major order: L unit lower block bidiagonal (L_k), U upper block
// bidiagonal (D_k, S_{k,k+1}); S^T = U^T L^T for the adjoint.  The
// off-diagonal blocks S_{k,k+1} = M_{k,k+1} A_b + K_{k,k+1} B_b are applied
// through the banded time matrices.  Lane j < nq owns row j of every block.
__global__ void __launch_bounds__(64) k_block_solve(const BlockDesc *__restrict__ bds) {
  constexpr int MAXQ = 64;
  __shared__ double s_v[MAXQ], s_u[MAXQ];
  const BlockDesc &B = cref(bds, blockIdx.x);
  const KernelTables &KT = cref(B.kt, 0);
  const int lane = threadIdx.x;
  const int nq = B.nq, nx = B.nx;
  const bool tr = B.transpose != 0;
  const gptr<const double> Ah = to_g(KT.A[B.b]), Bh = to_g(KT.B[B.b]), Al = to_g(KT.Alo[B.b]),
                          Bl = to_g(KT.Blo[B.b]);
  double *b0 = B.work, *res = b0 + (long long)nq * nx, *tmp = res + (long long)nq * nx;
  auto at = [&](int i, int k) -> long long { return (long long)i * nx + k; };
  // this lane's entries of the banded time matrices (its row of A and B, or
  // its column for the transpose), the same at every spatial block: read
  // once here instead of once per block and sweep (each read a round trip
  // on the sweep's sequential path)
  double tA[5], tB[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    const int off = o - 2, i = lane + off;
    const bool ok = lane < nq && i >= 0 && i < nq;
    const int e = ok ? (tr ? i * 5 + 2 - off : lane * 5 + off + 2) : 0;
    const double a = Ah[e], b = Bh[e];
    tA[o] = ok ? a : 0.0;
    tB[o] = ok ? b : 0.0;
  }
  // (T v)_lane for the banded time matrix T (A or B, high parts), T or T^T,
  // terms in the order off = -2..2
  auto band = [&](const double (&t)[5], const double *v) -> double {
    double acc = 0.0;
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int i = lane + o - 2;
      if (i < 0 || i >= nq) continue;
      acc += t[o] * v[i];
    }
    return acc;
  };
  // x <- op(S)^{-1} r (r read from R, result into X, may add); returns max |x|
  auto apply = [&](const double *R, double *X, bool add) -> double {
    double xm = 0.0;
    if (!tr) {
      // L y = r: y_k = r_k - L_k y_{k-1}   (y stored in tmp)
      for (int k = 0; k < nx; ++k) {
        double y = 0.0;
        if (lane < nq) {
          y = R[at(lane, k)];
          if (k > 0) {
            const double *Lk = B.Lf + ((long long)k * nq + lane) * nq;
            for (int i = 0; i < nq; ++i) y -= Lk[i] * s_v[i];
          }
        }
        __syncthreads();
        if (lane < nq) {
          s_v[lane] = y;
          tmp[at(lane, k)] = y;
        }
        __syncthreads();
      }
      // U x = y: x_k = D_k^{-1} (y_k - S_{k,k+1} x_{k+1})
      for (int k = nx - 1; k >= 0; --k) {
        if (lane < nq) {
          double w = tmp[at(lane, k)];
          if (k + 1 < nx)
            w -= B.mk[kSpaceStride * k + 1] * band(tA, s_v) +
                 B.mk[kSpaceStride * k + 3] * band(tB, s_v);
          s_u[lane] = w;
        }
        __syncthreads();
        double x = 0.0;
        if (lane < nq) {
          const double *Dk = B.Dinv + ((long long)k * nq + lane) * nq;
          for (int i = 0; i < nq; ++i) x += Dk[i] * s_u[i];
        }
        __syncthreads();
        if (lane < nq) {
          s_v[lane] = x;
          const double o = add ? X[at(lane, k)] + x : x;
          X[at(lane, k)] = o;
          xm = fmax(xm, fabs(x));
        }
        __syncthreads();
      }
    } else {
      // U^T w = r: w_k = D_k^{-T} (r_k - S_{k-1,k}^T w_{k-1})   (w in tmp)
      for (int k = 0; k < nx; ++k) {
        if (lane < nq) {
          double w = R[at(lane, k)];
          if (k > 0)
            w -= B.mk[kSpaceStride * (k - 1) + 1] * band(tA, s_v) +
                 B.mk[kSpaceStride * (k - 1) + 3] * band(tB, s_v);
          s_u[lane] = w;
        }
        __syncthreads();
        double x = 0.0;
        if (lane < nq)
          for (int i = 0; i < nq; ++i) x += B.Dinv[((long long)k * nq + i) * nq + lane] * s_u[i];
        __syncthreads();
        if (lane < nq) {
          s_v[lane] = x;
          tmp[at(lane, k)] = x;
        }
        __syncthreads();
      }
      // L^T z = w: z_k = w_k - L_{k+1}^T z_{k+1}
      for (int k = nx - 1; k >= 0; --k) {
        double z = 0.0;
        if (lane < nq) {
          z = tmp[at(lane, k)];
          if (k + 1 < nx) {
            const double *Lk = B.Lf + (long long)(k + 1) * nq * nq;
            for (int i = 0; i < nq; ++i) z -= Lk[(long long)i * nq + lane] * s_v[i];
          }
        }
        __syncthreads();
        if (lane < nq) {
          s_v[lane] = z;
          const double o = add ? X[at(lane, k)] + z : z;
          X[at(lane, k)] = o;
          xm = fmax(xm, fabs(z));
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int dlt = 32; dlt >= 1; dlt >>= 1) xm = fmax(xm, __shfl_xor(xm, dlt));
    return xm;
  };
  // b - op(S) x, every product and sum in double-double (time matrices and
  // K as hi+lo, M in double); also returns max |x|
  auto residual = [&](const double *X, double *Rout) -> double {
#pragma clang fp contract(off)
    double xmax = 0.0;
    for (long long e = lane; e < (long long)nq * nx; e += 64) {
      const int i = (int)(e / nx), k = (int)(e - (long long)i * nx);
      dd acc = {b0[e], 0.0};
      xmax = fmax(xmax, fabs(X[e]));
      for (int off = -2; off <= 2; ++off) {
        const int ii = i + off;
        if (ii < 0 || ii >= nq) continue;
        // spatial products (M x)_k and (K x)_k of row ii, in double-double
        dd ym = {0.0, 0.0}, yk = {0.0, 0.0};
        for (int sft = -1; sft <= 1; ++sft) {
          const int kk = k + sft;
          if (kk < 0 || kk >= nx) continue;
          const int lo = sft < 0 ? kk : k;  // M, K symmetric tridiagonal
          const double *e = B.mk + kSpaceStride * (sft == 0 ? k : lo) + (sft == 0 ? 0 : 1);
          const double x = X[at(ii, kk)];
          ym = dd_add(ym, two_prod(e[0], x));
          yk = dd_add(yk, two_prod(e[2], x));
          yk = dd_add(yk, dd{e[4] * x, 0.0});
        }
        const int r = tr ? ii : i, c = tr ? 2 - off : off + 2;
        const dd ta = dd_mul(dd{Ah[r * 5 + c], Al[r * 5 + c]}, ym);
        const dd tb = dd_mul(dd{Bh[r * 5 + c], Bl[r * 5 + c]}, yk);
        acc = dd_add(acc, dd{-ta.h, -ta.l});
        acc = dd_add(acc, dd{-tb.h, -tb.l});
      }
      Rout[e] = acc.h + acc.l;
    }
#pragma unroll
    for (int dlt = 32; dlt >= 1; dlt >>= 1) xmax = fmax(xmax, __shfl_xor(xmax, dlt));
    __syncthreads();
    return xmax;
  };
  for (long long e = lane; e < (long long)nq * nx; e += 64) b0[e] = B.in[e];
  __syncthreads();
  apply(b0, B.out, false);
  for (int it = 0; it < B.refine; ++it) {
    const double xmax = residual(B.out, res);
    const double dmax = apply(res, B.out, true);
    if (dmax <= 1e-15 * xmax) break;
  }
}

// File-scope scratch of sg_solve_static.  In host code `scratch` names a
// host-side stand-in, not device memory: host code uses only the address
// that static_scratch looks up.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

hipError_t static_scratch(double **ptr) {
  static std::mutex mu;
  static std::map<int, double *> addr;  // per device
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, static_cast<double *>(p)).first;
  }
  *ptr = it->second;
  return hipSuccess;
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

// tile side and slabs per batch (2-D, 1-D); the plan's time chunks are
// multiples of 8 slabs
// (measured on the 2-D level-10 workload: restriction is fastest with one
// slab per batch, prolongation with four; both are bound by the latency
// that their two resident waves per SIMD can hide)
#ifndef SG_TB2
#define SG_TB2 1
#endif
#ifndef SG_TB2P
#define SG_TB2P 4
#endif
constexpr int kTS2 = 32, kTB2 = SG_TB2, kTB2P = SG_TB2P, kTS1 = 256, kTB1 = 8, kNT = 256;

hipError_t launch_restrict(const RestrictArgs &a, hipStream_t s) {
  const int nt = a.g.d == 2 ? a.g.ntile * a.g.ntile : a.g.ntile;
  dim3 grid(nt, a.g.nchunk);
  const bool two = a.ch[(a.g.J - 1) * 2 + 1].active != 0;
#define SG_RESTRICT(D, TS, TB, ST, NC)                                                     \
  hipLaunchKernelGGL((k_restrict<D, TS, TB, kNT, ST, NC>), grid, dim3(kNT), 0, s, a)
#define SG_RESTRICT_W(ST, NC) \
  hipLaunchKernelGGL((k_restrict_w<ST, NC>), gridw, dim3(256), 0, s, a)
  if (a.g.d == 2 && a.g.TS == 16) {
    const int ng = (a.g.ntile + 1) / 2;
    dim3 gridw(ng * ng, a.g.nchunk);
    if (a.stencil) {
      if (two) SG_RESTRICT_W(1, 2); else SG_RESTRICT_W(1, 1);
    } else {
      if (two) SG_RESTRICT_W(0, 2); else SG_RESTRICT_W(0, 1);
    }
  } else if (a.g.d == 2) {
    if (a.stencil) {
      if (two) SG_RESTRICT(2, kTS2, kTB2, 1, 2); else SG_RESTRICT(2, kTS2, kTB2, 1, 1);
    } else {
      if (two) SG_RESTRICT(2, kTS2, kTB2, 0, 2); else SG_RESTRICT(2, kTS2, kTB2, 0, 1);
    }
  } else {
    if (a.stencil) {
      if (two) SG_RESTRICT(1, kTS1, kTB1, 1, 2); else SG_RESTRICT(1, kTS1, kTB1, 1, 1);
    } else {
      if (two) SG_RESTRICT(1, kTS1, kTB1, 0, 2); else SG_RESTRICT(1, kTS1, kTB1, 0, 1);
    }
  }
#undef SG_RESTRICT
#undef SG_RESTRICT_W
  return hipGetLastError();
}

hipError_t launch_reduce(const Geometry &g, const Channel *ch, const double *part,
                         const WorkItem *items, int nitems, long long total,
                         hipStream_t s) {
  if (total == 0) return hipSuccess;
  if (g.d == 2 && g.TS == 16)
    hipLaunchKernelGGL((k_reduce<2, 16>), dim3(blocks_for(total, 256)), dim3(256), 0, s,
                       g, ch, part, items, nitems, total);
  else if (g.d == 2)
    hipLaunchKernelGGL((k_reduce<2, kTS2>), dim3(blocks_for(total, 256)), dim3(256), 0, s,
                       g, ch, part, items, nitems, total);
  else
    hipLaunchKernelGGL((k_reduce<1, kTS1>), dim3(blocks_for(total, 256)), dim3(256), 0, s,
                       g, ch, part, items, nitems, total);
  return hipGetLastError();
}

hipError_t launch_coarse_pyramid(const Geometry &g, const double *cp, double *SL,
                                 hipStream_t s) {
  if (g.A0 <= 1) return hipSuccess;
  if (g.d == 2)
    hipLaunchKernelGGL(k_coarse_pyramid<2>, dim3(g.ntf), dim3(256), 0, s, g, cp, SL);
  else
    hipLaunchKernelGGL(k_coarse_pyramid<1>, dim3(g.ntf), dim3(256), 0, s, g, cp, SL);
  return hipGetLastError();
}

hipError_t launch_coarse_restrict(const Geometry &g, const Channel *ch, const double *SL,
                                  const WorkItem *items, int nitems, long long total,
                                  hipStream_t s) {
  if (total == 0) return hipSuccess;
  if (g.d == 2)
    hipLaunchKernelGGL(k_coarse_restrict<2>, dim3(blocks_for(total, 128)), dim3(128), 0, s,
                       g, ch, SL, items, nitems, total);
  else
    hipLaunchKernelGGL(k_coarse_restrict<1>, dim3(blocks_for(total, 128)), dim3(128), 0, s,
                       g, ch, SL, items, nitems, total);
  return hipGetLastError();
}

hipError_t launch_prolong_coarse(const Geometry &g, const Channel *ch, double *C, int,
                                 hipStream_t s) {
  // one block per slab
  if (g.d == 2)
    hipLaunchKernelGGL(k_prolong_coarse<2>, dim3(g.ntf), dim3(256), 0, s, g, ch, C);
  else
    hipLaunchKernelGGL(k_prolong_coarse<1>, dim3(g.ntf), dim3(256), 0, s, g, ch, C);
  return hipGetLastError();
}

hipError_t launch_prolong(const ProlongArgs &a, hipStream_t s) {
  const int nt = a.g.d == 2 ? a.g.ntile * a.g.ntile : a.g.ntile;
  dim3 grid(nt, a.g.nchunk);
  const bool two = a.ch[(a.g.J - 1) * 2 + 1].active != 0;
#define SG_PROLONG(D, TS, TB, MO, NC)                                                      \
  hipLaunchKernelGGL((k_prolong<D, TS, TB, kNT, MO, NC>), grid, dim3(kNT), 0, s, a)
  if (a.g.d == 2 && a.g.TS == 16) {
    if (two || a.taps == nullptr) return hipErrorInvalidValue;  // one finest channel only
    const int ngx = (a.g.ntile + 3) / 4;  // four tiles side by side per workgroup
    dim3 gridw(ngx * a.g.ntile, a.g.nchunk);
    if (a.stencil)
      hipLaunchKernelGGL(k_prolong_wm, gridw, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(k_prolong_w, gridw, dim3(256), 0, s, a);
  } else if (a.g.d == 2) {
    if (a.stencil) {
      if (two) SG_PROLONG(2, kTS2, kTB2P, 1, 2); else SG_PROLONG(2, kTS2, kTB2P, 1, 1);
    } else {
      if (two) SG_PROLONG(2, kTS2, kTB2P, 0, 2); else SG_PROLONG(2, kTS2, kTB2P, 0, 1);
    }
  } else {
    if (a.stencil) {
      if (two) SG_PROLONG(1, kTS1, kTB1, 1, 2); else SG_PROLONG(1, kTS1, kTB1, 1, 1);
    } else {
      if (two) SG_PROLONG(1, kTS1, kTB1, 0, 2); else SG_PROLONG(1, kTS1, kTB1, 0, 1);
    }
  }
#undef SG_PROLONG
  return hipGetLastError();
}

hipError_t launch_energy(int d, int N, const double *ce, double hx, double hy, const double *W,
                         const double *Ut, int K, int nblk, double *part, double *E,
                         hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const dim3 grid(nblk, K);
  if (d == 2)
    hipLaunchKernelGGL(k_energy_part<2>, grid, dim3(256), 0, s, N, ce, hx, hy, W, Ut, part);
  else
    hipLaunchKernelGGL(k_energy_part<1>, grid, dim3(256), 0, s, N, ce, hx, hy, W, Ut, part);
  hipLaunchKernelGGL(k_energy_sum, dim3(K), dim3(64), 0, s, K, nblk, part, E);
  return hipGetLastError();
}

hipError_t launch_energy_w(const ProlongArgs &a, const TapEntry *taps_d, const double *coarse_d,
                           const double *ce, double hx, double hy, double *part, int K,
                           int ntile2, double *E, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  if (a.g.d != 2 || a.g.TS != 16 || a.taps == nullptr || taps_d == nullptr ||
      a.g.ntile * a.g.ntile != ntile2 || a.g.ntf != K)
    return hipErrorInvalidValue;
  const int ngx = (a.g.ntile + 3) / 4;  // four tiles side by side per workgroup
  hipLaunchKernelGGL(k_energy_w, dim3(ngx * a.g.ntile, a.g.nchunk), dim3(256), 0, s, a, taps_d,
                     coarse_d, ce, hx, hy, part);
  hipLaunchKernelGGL(k_energy_sum, dim3(K), dim3(64), 0, s, K, ntile2, part, E);
  return hipGetLastError();
}

hipError_t launch_l2(int d, int N, double hx, double hy, const double *W, const double *uq,
                     int K, int nblk, double *part, const double *wt, double *out,
                     hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const dim3 grid(nblk, K);
  if (d == 2)
    hipLaunchKernelGGL(k_l2_part<2>, grid, dim3(256), 0, s, N, hx, hy, W, uq, part);
  else
    hipLaunchKernelGGL(k_l2_part<1>, grid, dim3(256), 0, s, N, hx, hy, W, uq, part);
  hipLaunchKernelGGL(k_l2_sum, dim3(1), dim3(64), 0, s, K, nblk, part, wt, out);
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

hipError_t launch_post_load(const CompDesc *cd, int ncomp, long long total, hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_post_load, dim3(blocks_for(total, 256)), dim3(256), 0, s, cd, ncomp,
                     total);
  return hipGetLastError();
}

hipError_t launch_post_adjoint(const CompDesc *cd, int ncomp, long long total, hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_post_adjoint, dim3(blocks_for(total, 256)), dim3(256), 0, s, cd,
                     ncomp, total);
  return hipGetLastError();
}

hipError_t launch_adjoint_fields(const LevelDesc *ld, int nlev, long long total,
                                 hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adjoint_fields, dim3(blocks_for(total, 256)), dim3(256), 0, s, ld,
                     nlev, total);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmDesc *descs, int ndesc, int total_tiles, int fold,
                       hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  if (fold == 1)
    hipLaunchKernelGGL(k_gemm<1>, dim3(total_tiles), dim3(kGemmThreads), 0, s, descs, ndesc);
  else if (fold == 2)
    hipLaunchKernelGGL(k_gemm<2>, dim3(total_tiles), dim3(kGemmThreads), 0, s, descs, ndesc);
  else if (fold == 3)
    hipLaunchKernelGGL(k_gemm<3>, dim3(total_tiles), dim3(kGemmThreads), 0, s, descs, ndesc);
  else if (fold == 4)
    hipLaunchKernelGGL(k_gemm<4>, dim3(total_tiles), dim3(kGemmThreads), 0, s, descs, ndesc);
  else
    hipLaunchKernelGGL(k_gemm<0>, dim3(total_tiles), dim3(kGemmThreads), 0, s, descs, ndesc);
  return hipGetLastError();
}

hipError_t launch_time_factor(const SolveDesc *sd, int nsd, long long total, hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_factor, dim3(blocks_for(total, 64)), dim3(64), 0, s, sd, nsd,
                     total);
  return hipGetLastError();
}

hipError_t launch_time_solve(const SolveDesc *sd, int nsd, long long total, int transpose,
                             hipStream_t s) {
  if (total == 0) return hipSuccess;
  if (transpose)
    hipLaunchKernelGGL(k_time_solve<1>, dim3(blocks_for(total, 64)), dim3(64), 0, s, sd, nsd,
                       total);
  else
    hipLaunchKernelGGL(k_time_solve<0>, dim3(blocks_for(total, 64)), dim3(64), 0, s, sd, nsd,
                       total);
  return hipGetLastError();
}

hipError_t launch_block_solve(const BlockDesc *bd, int nbd, hipStream_t s) {
  if (nbd == 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_solve, dim3(nbd), dim3(64), 0, s, bd);
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

// ---- launches of many problems -----------------------------------------------

hipError_t launch_restrict_many(const RestrictArgs &a, const ManyLaunch &M, int blocks,
                                hipStream_t s) {
  if (blocks <= 0 || M.n <= 0) return hipSuccess;
  const bool two = a.ch[(a.g.J - 1) * 2 + 1].active != 0;
  const dim3 grid(blocks);
#define SG_RM(D, TS, TB, ST, NC) \
  hipLaunchKernelGGL((k_restrict_many<D, TS, TB, kNT, ST, NC>), grid, dim3(kNT), 0, s, M)
#define SG_RMW(ST, NC) hipLaunchKernelGGL((k_restrict_w_many<ST, NC>), grid, dim3(256), 0, s, M)
  if (a.g.d == 2 && a.g.TS == 16) {
    if (a.stencil) {
      if (two) SG_RMW(1, 2); else SG_RMW(1, 1);
    } else {
      if (two) SG_RMW(0, 2); else SG_RMW(0, 1);
    }
  } else if (a.g.d == 2) {
    if (a.stencil) {
      if (two) SG_RM(2, kTS2, kTB2, 1, 2); else SG_RM(2, kTS2, kTB2, 1, 1);
    } else {
      if (two) SG_RM(2, kTS2, kTB2, 0, 2); else SG_RM(2, kTS2, kTB2, 0, 1);
    }
  } else {
    if (a.stencil) {
      if (two) SG_RM(1, kTS1, kTB1, 1, 2); else SG_RM(1, kTS1, kTB1, 1, 1);
    } else {
      if (two) SG_RM(1, kTS1, kTB1, 0, 2); else SG_RM(1, kTS1, kTB1, 0, 1);
    }
  }
#undef SG_RM
#undef SG_RMW
  return hipGetLastError();
}

hipError_t launch_prolong_many(const ProlongArgs &a, const ManyLaunch &M, int blocks,
                               hipStream_t s) {
  if (blocks <= 0 || M.n <= 0) return hipSuccess;
  const bool two = a.ch[(a.g.J - 1) * 2 + 1].active != 0;
  const dim3 grid(blocks);
#define SG_PM(D, TS, TB, MO, NC) \
  hipLaunchKernelGGL((k_prolong_many<D, TS, TB, kNT, MO, NC>), grid, dim3(kNT), 0, s, M)
  if (a.g.d == 2 && a.g.TS == 16) {
    if (two || a.taps == nullptr) return hipErrorInvalidValue;  // one finest channel only
    if (a.stencil)
      hipLaunchKernelGGL(k_prolong_wm_many, grid, dim3(256), 0, s, M);
    else
      hipLaunchKernelGGL(k_prolong_w_many, grid, dim3(256), 0, s, M);
  } else if (a.g.d == 2) {
    if (a.stencil) {
      if (two) SG_PM(2, kTS2, kTB2P, 1, 2); else SG_PM(2, kTS2, kTB2P, 1, 1);
    } else {
      if (two) SG_PM(2, kTS2, kTB2P, 0, 2); else SG_PM(2, kTS2, kTB2P, 0, 1);
    }
  } else {
    if (a.stencil) {
      if (two) SG_PM(1, kTS1, kTB1, 1, 2); else SG_PM(1, kTS1, kTB1, 1, 1);
    } else {
      if (two) SG_PM(1, kTS1, kTB1, 0, 2); else SG_PM(1, kTS1, kTB1, 0, 1);
    }
  }
#undef SG_PM
  return hipGetLastError();
}

hipError_t launch_reduce_many(const Geometry &g, const ManyLaunch &M, int blocks,
                              hipStream_t s) {
  if (blocks <= 0 || M.n <= 0) return hipSuccess;
  if (g.d == 2 && g.TS == 16)
    hipLaunchKernelGGL((k_reduce_many<2, 16>), dim3(blocks), dim3(256), 0, s, M);
  else if (g.d == 2)
    hipLaunchKernelGGL((k_reduce_many<2, kTS2>), dim3(blocks), dim3(256), 0, s, M);
  else
    hipLaunchKernelGGL((k_reduce_many<1, kTS1>), dim3(blocks), dim3(256), 0, s, M);
  return hipGetLastError();
}

hipError_t launch_coarse_pyramid_many(int d, const ManyLaunch &M, int blocks, hipStream_t s) {
  if (blocks <= 0 || M.n <= 0) return hipSuccess;
  if (d == 2)
    hipLaunchKernelGGL(k_coarse_pyramid_many<2>, dim3(blocks), dim3(256), 0, s, M);
  else
    hipLaunchKernelGGL(k_coarse_pyramid_many<1>, dim3(blocks), dim3(256), 0, s, M);
  return hipGetLastError();
}

hipError_t launch_coarse_restrict_many(int d, const ManyLaunch &M, int blocks, hipStream_t s) {
  if (blocks <= 0 || M.n <= 0) return hipSuccess;
  if (d == 2)
    hipLaunchKernelGGL(k_coarse_restrict_many<2>, dim3(blocks), dim3(256), 0, s, M);
  else
    hipLaunchKernelGGL(k_coarse_restrict_many<1>, dim3(blocks), dim3(256), 0, s, M);
  return hipGetLastError();
}

hipError_t launch_prolong_coarse_many(int d, const ManyLaunch &M, int blocks, hipStream_t s) {
  if (blocks <= 0 || M.n <= 0) return hipSuccess;
  if (d == 2)
    hipLaunchKernelGGL(k_prolong_coarse_many<2>, dim3(blocks), dim3(256), 0, s, M);
  else
    hipLaunchKernelGGL(k_prolong_coarse_many<1>, dim3(blocks), dim3(256), 0, s, M);
  return hipGetLastError();
}

hipError_t launch_fine_stencils_many(int d, const ManyLaunch &M, int blocks, hipStream_t s) {
  if (blocks <= 0 || M.n <= 0) return hipSuccess;
  if (d == 2)
    hipLaunchKernelGGL(k_fine_stencils_many<2>, dim3(blocks), dim3(256), 0, s, M);
  else
    hipLaunchKernelGGL(k_fine_stencils_many<1>, dim3(blocks), dim3(256), 0, s, M);
  return hipGetLastError();
}

}  // namespace sg
