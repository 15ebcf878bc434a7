// 2-D variable-speed components of short time levels (gfx950, FP64).
//
// The component system S = A (x) M + B (x) K(c) of eq. (9) is diagonalised in
// time (B^{-1} A = V diag(lam) V^{-1}, host tables), which leaves one complex
// shifted spatial system per eigenvalue,
//     (lam M + K(c)) w = r,     M, K(c) the Q1 mass and stiffness,
// one of each conjugate pair.  For lam real (positive at these levels) the
// system is symmetric positive definite; otherwise its imaginary part is a
// definite multiple of M.  Each system is solved directly:
//   * Omega is cut into the ns strips of wave-speed blocks along y.  Inside
//     strip k, c depends on x only, so the strip operator is
//     My0 (x) (lam Mx + Kx^k) + Ky0 (x) Mx^k with the constant-coefficient
//     1-D matrices My0, Ky0 of the strip's m interior rows; the orthonormal
//     sine transform along y diagonalises them (mu_l, nu_l) and leaves one
//     tridiagonal system in x per mode l:
//         T_{k,l} = mu_l (lam Mx + Kx^k) + nu_l Mx^k.
//   * The ni = ns - 1 interface rows between strips carry the Schur
//     complement S_G (block tridiagonal in the interfaces, dense blocks of
//     n x n), formed and inverted at assembly.
// Solve: strip solves with the interface rows held at zero, the interface
// right-hand side, x_G = S_G^{-1} g, and a correction of the strip solutions
// by the interface values (one more tridiagonal solve per mode).
//
// Complex values are interleaved (re, im) doubles.  The strip sine transforms
// run as GEMMs on the matrix cores (launch_gemm, lists built by the plan).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "gmem.hpp"

namespace sg {

namespace {

struct cx {
  double r, i;
};
__device__ __forceinline__ cx cadd(cx a, cx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cx csub(cx a, cx b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cx cmul(cx a, cx b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
__device__ __forceinline__ cx cscl(cx a, double s) { return {a.r * s, a.i * s}; }
// 1 / a with scaling against overflow
__device__ __forceinline__ cx crcp(cx a) {
  const double s = fmax(fabs(a.r), fabs(a.i));
  const double ar = a.r / s, ai = a.i / s;
  const double d = (ar * ar + ai * ai) * s;
  return {ar / d, -ai / d};
}
__device__ __forceinline__ cx cld(const double *p) { return {p[0], p[1]}; }
__device__ __forceinline__ void cst(double *p, cx v) {
  p[0] = v.r;
  p[1] = v.i;
}

__device__ __forceinline__ long long gid64() {
  return (long long)blockIdx.x * blockDim.x + threadIdx.x;
}

enum Field { kNode, kTri, kEdge, kIf, kGemv };

__device__ __forceinline__ long long start_of(const FdmDesc &D, int f) {
  switch (f) {
    case kNode: return D.node0;
    case kTri: return D.tri0;
    case kEdge: return D.edge0;
    case kIf: return D.if0;
    default: return D.gemv0;
  }
}

// last descriptor whose start (of the given field) is <= g
__device__ __forceinline__ int find_fdm(const FdmDesc *d, int nd, long long g, int f) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start_of(d[mid], f) <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Row x of T_{k,l}(lam): diagonal dg and coupling of, between x and x + 1
// (zero at the last row).  Mx is the uniform P1 mass (2 hx / 3, hx / 6).
__device__ __forceinline__ void tri_row(const FdmDesc &D, int k, int l, cx lam, int x, cx &dg,
                                        cx &of) {
  const double mu = D.ym[l], nu = D.ym[D.m + l];
  const double *t = D.xt + (size_t)k * 4 * D.n;
  const double mxd = 2.0 * D.hx / 3.0, mxo = D.hx / 6.0;
  dg = {mu * (lam.r * mxd + t[x]) + nu * t[2 * D.n + x], mu * lam.i * mxd};
  if (x + 1 < D.n)
    of = {mu * (lam.r * mxo + t[D.n + x]) + nu * t[3 * D.n + x], mu * lam.i * mxo};
  else
    of = {0.0, 0.0};
}

// Row x of the coupling C_k = (hy/6)(lam Mx + Kx^k) - Mx^k / hy between the
// first (last) row of strip k and the interface row below (above) it.
__device__ __forceinline__ void cpl_row(const FdmDesc &D, int k, cx lam, int x, cx &dg,
                                        cx &of) {
  const double *t = D.xt + (size_t)k * 4 * D.n;
  const double a = D.hy / 6.0, b = 1.0 / D.hy;
  const double mxd = 2.0 * D.hx / 3.0, mxo = D.hx / 6.0;
  dg = {a * (lam.r * mxd + t[x]) - b * t[2 * D.n + x], a * lam.i * mxd};
  if (x + 1 < D.n)
    of = {a * (lam.r * mxo + t[D.n + x]) - b * t[3 * D.n + x], a * lam.i * mxo};
  else
    of = {0.0, 0.0};
}

// (C_k v)[x] for a complex row v of n entries
__device__ __forceinline__ cx cpl_apply(const FdmDesc &D, int k, cx lam, const double *v,
                                        int x) {
  cx dg, of;
  cpl_row(D, k, lam, x, dg, of);
  cx r = cmul(dg, cld(v + 2 * x));
  if (x + 1 < D.n) r = cadd(r, cmul(of, cld(v + 2 * (x + 1))));
  if (x > 0) {
    cx d2, o2;
    cpl_row(D, k, lam, x - 1, d2, o2);
    r = cadd(r, cmul(o2, cld(v + 2 * (x - 1))));
  }
  return r;
}

// Row x of the interface block D_r (interface r between strips r - 1 and r):
// each strip contributes (hy/3)(lam Mx + Kx^k) + Mx^k / hy.
__device__ __forceinline__ void dif_row(const FdmDesc &D, int r, cx lam, int x, cx &dg,
                                        cx &of) {
  const double a = D.hy / 3.0, b = 1.0 / D.hy;
  const double mxd = 2.0 * D.hx / 3.0, mxo = D.hx / 6.0;
  dg = {0.0, 0.0};
  of = {0.0, 0.0};
  for (int k = r - 1; k <= r; ++k) {
    const double *t = D.xt + (size_t)k * 4 * D.n;
    dg = cadd(dg, cx{a * (lam.r * mxd + t[x]) + b * t[2 * D.n + x], a * lam.i * mxd});
    if (x + 1 < D.n)
      of = cadd(of, cx{a * (lam.r * mxo + t[D.n + x]) + b * t[3 * D.n + x], a * lam.i * mxo});
  }
}

// factor planes of T_{k,l}: kInvD 1/d'_x (top-down LU pivot), kEll l_x (its
// multiplier), kInvB 1/d''_x (bottom-up pivot); each plane complex
// [u][k][x][l], so a sweep over x reads only the plane it needs, the modes l
// of a wave side by side
enum FacPlane { kInvD = 0, kEll = 1, kInvB = 2 };
__device__ __forceinline__ double *fac_at(const FdmDesc &D, int plane, int u, int k, int x,
                                          int l) {
  const size_t per = (size_t)D.nu * D.ns * D.n * D.m;
  return D.fac + 2 * (plane * per + (((size_t)u * D.ns + k) * D.n + x) * D.m + l);
}

// ---------------------------------------------------------------- solve ----

// X[u][node] = sum_j tin[u][j] in[j][node]  (u < nu <= kFdmMaxNu: the
// accumulators stay in registers)
__global__ void k_fdm_in(const FdmDesc *__restrict__ ds, int nd, long long total) {
  const long long g = gid64();
  if (g >= total) return;
  const FdmDesc &D = cref(ds, find_fdm(ds, nd, g, kNode));
  const long long node = g - D.node0, nn = (long long)D.n * D.n;
  const int nq = D.nq, nu = D.nu;
  cx acc[kFdmMaxNu];
#pragma unroll
  for (int u = 0; u < kFdmMaxNu; ++u) acc[u] = {0.0, 0.0};
  for (int j = 0; j < nq; ++j) {
    const double v = D.in[(long long)j * nn + node];
#pragma unroll
    for (int u = 0; u < kFdmMaxNu; ++u)
      if (u < nu) acc[u] = cadd(acc[u], cscl(cld(D.tin + 2 * ((size_t)u * nq + j)), v));
  }
#pragma unroll
  for (int u = 0; u < kFdmMaxNu; ++u)
    if (u < nu) cst(D.X + 2 * ((long long)u * nn + node), acc[u]);
}

// out[j][node] = Re sum_u tout[j][u] w_u[node], w from X (strip rows) or Xg
// (interface rows)
__global__ void k_fdm_out(const FdmDesc *__restrict__ ds, int nd, long long total) {
  const long long g = gid64();
  if (g >= total) return;
  const FdmDesc &D = cref(ds, find_fdm(ds, nd, g, kNode));
  const long long node = g - D.node0, nn = (long long)D.n * D.n;
  const int y = (int)(node / D.n), x = (int)(node - (long long)y * D.n);
  const bool iface = (y + 1) % (D.m + 1) == 0;
  const int r = (y + 1) / (D.m + 1);  // 1-based interface index
  const int nu = D.nu;
  cx w[kFdmMaxNu];
#pragma unroll
  for (int u = 0; u < kFdmMaxNu; ++u)
    w[u] = u >= nu ? cx{0.0, 0.0}
           : iface ? cld(D.Xg + 2 * (((size_t)u * D.ni + r - 1) * D.n + x))
                   : cld(D.X + 2 * ((long long)u * nn + node));
  for (int j = 0; j < D.nq; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kFdmMaxNu; ++u)
      if (u < nu) {
        const cx t = cld(D.tout + 2 * ((size_t)j * nu + u));
        acc += t.r * w[u].r - t.i * w[u].i;
      }
    D.out[(long long)j * nn + node] = acc;
  }
}

// One thread per (u, k, l): the tridiagonal solve along x of mode l of
// strip k, in place on row (k (m+1) + l) of Y.
//   correction 0: Y <- T^{-1} Y
//   correction 1: Y <- Y - T^{-1} (s_l(first) C_k x_lo + s_l(last) C_k x_hi),
//                 x_lo / x_hi the interface solutions below / above the strip
//                 (the forward sweep is kept in the same row of X, whose strip
//                 rows are free at this point)
// Both sweeps run in chunks of FCH rows: the chunk's operands are loaded into
// registers first (independent loads in flight together), then the
// recurrence runs on registers.
template <int FCH>
__global__ void __launch_bounds__(64) k_fdm_tri(const FdmDesc *__restrict__ ds, int nd,
                                                long long total, int correction) {
  const long long g = gid64();
  if (g >= total) return;
  const FdmDesc &D = cref(ds, find_fdm(ds, nd, g, kTri));
  const int t = (int)(g - D.tri0);
  const int l = t % D.m, k = (t / D.m) % D.ns, u = t / (D.m * D.ns);
  const cx lam = cld(D.lam + 2 * u);
  const int n = D.n, m = D.m;
  // the strip's transformed values, mode-fastest: (x, re/im, l) at
  // (2 x + re/im) m + l from the strip's start (the forward sweep of the
  // correction keeps its values in the same layout in X, whose strip rows
  // are free at this point); a wave's lanes read side by side
  const long long strip = 2 * (((long long)u * n + (long long)k * (m + 1)) * n);
  double *Yr = D.Y + strip + l;
  double *Wr = (correction ? D.X + strip : D.Y + strip) + l;
  auto ldv = [&](const double *b, int x) -> cx {
    return {b[2LL * x * m], b[(2LL * x + 1) * m]};
  };
  auto stv = [&](double *b, int x, cx v) {
    b[2LL * x * m] = v.r;
    b[(2LL * x + 1) * m] = v.i;
  };
  const double *xlo = nullptr, *xhi = nullptr;
  double s0 = 0.0, s1 = 0.0;
  if (correction) {
    if (D.ni == 0) return;
    s0 = D.ym[2 * D.m + l];
    s1 = (l & 1) ? -s0 : s0;  // s_l(last) = (-1)^l s_l(first)
    if (k >= 1) xlo = D.Xg + 2 * (((size_t)u * D.ni + (k - 1)) * n);
    if (k + 1 <= D.ni) xhi = D.Xg + 2 * (((size_t)u * D.ni + k) * n);
  }
  auto rhs = [&](int x) -> cx {
    if (!correction) return ldv(Yr, x);
    cx r = {0.0, 0.0};
    if (xlo) r = cadd(r, cscl(cpl_apply(D, k, lam, xlo, x), s0));
    if (xhi) r = cadd(r, cscl(cpl_apply(D, k, lam, xhi, x), s1));
    return r;
  };
  // forward sweep: y_x = r_x - l_x y_{x-1} (l_0 = 0)
  cx prev = {0.0, 0.0};
  for (int x0 = 0; x0 < n; x0 += FCH) {
    cx r[FCH], el[FCH];
#pragma unroll
    for (int c = 0; c < FCH; ++c) {
      const int x = min(x0 + c, n - 1);
      r[c] = rhs(x);
      el[c] = cld(fac_at(D, kEll, u, k, x, l));
    }
#pragma unroll
    for (int c = 0; c < FCH; ++c) {
      if (x0 + c < n) {
        prev = csub(r[c], cmul(el[c], prev));
        stv(Wr, x0 + c, prev);
      }
    }
  }
  // back substitution: z_x = (y_x - of_x z_{x+1}) / d'_x, chunks from the top
  cx z = {0.0, 0.0};
  for (int x1 = n - 1; x1 >= 0; x1 -= FCH) {
    cx w[FCH], iv[FCH], of[FCH], yo[FCH];
#pragma unroll
    for (int c = 0; c < FCH; ++c) {
      const int x = max(x1 - c, 0);
      w[c] = ldv(Wr, x);
      iv[c] = cld(fac_at(D, kInvD, u, k, x, l));
      cx dg;
      tri_row(D, k, l, lam, x, dg, of[c]);
      if (correction) yo[c] = ldv(Yr, x);
    }
#pragma unroll
    for (int c = 0; c < FCH; ++c) {
      const int x = x1 - c;
      if (x >= 0) {
        z = cmul(csub(w[c], cmul(of[c], z)), iv[c]);
        stv(Yr, x, correction ? csub(yo[c], z) : z);
      }
    }
  }
}

// E[u][k][0|1][x] = the strip solution at the strip's first / last row:
// the inverse sine transform restricted to those rows
__global__ void k_fdm_edge(const FdmDesc *__restrict__ ds, int nd, long long total) {
  // 16 lanes per (u, k, x): the strip's values at x are mode-fastest (see
  // k_fdm_tri), so lane j sums the modes l = j, j + 16, ... (coalesced) and
  // the 16 partial sums are combined by a butterfly within the lane group
  constexpr int G = 16;
  const long long g = gid64() / G;
  const int j = (int)(threadIdx.x % G);
  if (g >= total) return;  // whole lane groups
  const FdmDesc &D = cref(ds, find_fdm(ds, nd, g, kEdge));
  const int t = (int)(g - D.edge0);
  const int x = t % D.n, k = (t / D.n) % D.ns, u = t / (D.n * D.ns);
  const double *Y = D.Y + 2 * (((long long)u * D.n + (long long)k * (D.m + 1)) * D.n) +
                    2LL * x * D.m;
  cx f = {0.0, 0.0}, la = {0.0, 0.0};
  for (int l = j; l < D.m; l += G) {
    const double s = D.ym[2 * D.m + l];
    const cx v = cscl(cx{Y[l], Y[D.m + l]}, s);
    f = cadd(f, v);
    la = (l & 1) ? csub(la, v) : cadd(la, v);
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) {
    f.r += __shfl_xor(f.r, o);
    f.i += __shfl_xor(f.i, o);
    la.r += __shfl_xor(la.r, o);
    la.i += __shfl_xor(la.i, o);
  }
  if (j != 0) return;
  double *E = D.E + 2 * ((((size_t)u * D.ns + k) * 2) * D.n + x);
  cst(E, f);
  cst(E + 2 * D.n, la);
}

// G[u][r-1][x] = r_u(interface row r) - C_{r-1} (strip r-1 at its last row)
//                - C_r (strip r at its first row)
__global__ void k_fdm_iface(const FdmDesc *__restrict__ ds, int nd, long long total) {
  const long long g = gid64();
  if (g >= total) return;
  const FdmDesc &D = cref(ds, find_fdm(ds, nd, g, kIf));
  const int t = (int)(g - D.if0);
  const int x = t % D.n, r = (t / D.n) % D.ni + 1, u = t / (D.n * D.ni);
  const cx lam = cld(D.lam + 2 * u);
  const int y = r * (D.m + 1) - 1;
  cx v = cld(D.X + 2 * (((long long)u * D.n + y) * D.n + x));
  const double *Eb = D.E + 2 * ((((size_t)u * D.ns + (r - 1)) * 2 + 1) * D.n);  // last row, below
  const double *Ea = D.E + 2 * ((((size_t)u * D.ns + r) * 2 + 0) * D.n);        // first row, above
  v = csub(v, cpl_apply(D, r - 1, lam, Eb, x));
  v = csub(v, cpl_apply(D, r, lam, Ea, x));
  cst(D.G + 2 * (((size_t)u * D.ni + (r - 1)) * D.n + x), v);
}

// Xg[u] = Sinv[u] G[u]: one wave per output row
__global__ void __launch_bounds__(256) k_fdm_gemv(const FdmDesc *__restrict__ ds, int nd,
                                                  long long total) {
  const long long w = gid64() >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= total) return;
  const FdmDesc &D = cref(ds, find_fdm(ds, nd, w, kGemv));
  const long long rw = w - D.gemv0;
  const long long NG = (long long)D.ni * D.n;
  const long long u = rw / NG, rho = rw - u * NG;
  const double *Srow = D.Sinv + 2 * ((u * NG + rho) * NG);
  const double *gv = D.G + 2 * (u * NG);
  double ar = 0.0, ai = 0.0;
  for (long long c = lane; c < NG; c += 64) {
    const double sr = Srow[2 * c], si = Srow[2 * c + 1];
    const double gr = gv[2 * c], gi = gv[2 * c + 1];
    ar += sr * gr - si * gi;
    ai += sr * gi + si * gr;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    ar += __shfl_xor(ar, o);
    ai += __shfl_xor(ai, o);
  }
  if (lane == 0) {
    double *o = D.Xg + 2 * (u * NG + rho);
    o[0] = ar;
    o[1] = ai;
  }
}

// ------------------------------------------------------------- assembly ----

// one thread per (u, k, l): top-down and bottom-up elimination of T_{k,l}
__global__ void k_fdm_factor(const FdmDesc D) {
  const long long g = gid64();
  if (g >= (long long)D.nu * D.ns * D.m) return;
  const int l = (int)(g % D.m), k = (int)((g / D.m) % D.ns), u = (int)(g / ((long long)D.m * D.ns));
  const cx lam = cld(D.lam + 2 * u);
  cx dg, of, ofp;
  tri_row(D, k, l, lam, 0, dg, of);
  cx inv = crcp(dg);
  cst(fac_at(D, kInvD, u, k, 0, l), inv);
  cst(fac_at(D, kEll, u, k, 0, l), cx{0.0, 0.0});
  for (int x = 1; x < D.n; ++x) {
    ofp = of;                      // coupling (x-1, x)
    tri_row(D, k, l, lam, x, dg, of);
    const cx ell = cmul(ofp, inv);  // l_x = of_{x-1} / d'_{x-1}
    inv = crcp(csub(dg, cmul(ell, ofp)));
    cst(fac_at(D, kInvD, u, k, x, l), inv);
    cst(fac_at(D, kEll, u, k, x, l), ell);
  }
  // bottom-up: d''_{n-1} = dg_{n-1}, d''_x = dg_x - of_x^2 / d''_{x+1}
  tri_row(D, k, l, lam, D.n - 1, dg, of);
  cx invb = crcp(dg);
  cst(fac_at(D, kInvB, u, k, D.n - 1, l), invb);
  for (int x = D.n - 2; x >= 0; --x) {
    tri_row(D, k, l, lam, x, dg, of);
    invb = crcp(csub(dg, cmul(cmul(of, of), invb)));
    cst(fac_at(D, kInvB, u, k, x, l), invb);
  }
}

// Strip Green's functions next to the interfaces, per group of modes:
//   P0[u][k][grp][x][j] = sum_{l in grp} s_l(first)^2 (T_{k,l}^{-1})[x][j],
//   P1[...]             = sum_{l in grp} s_l(first) s_l(last) (T_{k,l}^{-1})[x][j]
// (s_l(last)^2 = s_l(first)^2, so the last-row block equals the first-row
// one).  Column j of T^{-1} without scratch: its pivot entry is
// 1 / (dg_j - of_{j-1}^2 / d'_{j-1} - of_j^2 / d''_{j+1}); above it
// x_i = -of_i / d'_i x_{i+1}, below it x_i = -of_{i-1} / d''_i x_{i-1}.
__global__ void k_fdm_green(const FdmDesc D, int ngrp, double *P0, double *P1) {
  const long long g = gid64();
  const int n = D.n;
  if (g >= (long long)D.nu * D.ns * ngrp * n) return;
  const int j = (int)(g % n);
  const int grp = (int)((g / n) % ngrp);
  const int k = (int)((g / ((long long)n * ngrp)) % D.ns);
  const int u = (int)(g / ((long long)n * ngrp * D.ns));
  const cx lam = cld(D.lam + 2 * u);
  const int lpg = (D.m + ngrp - 1) / ngrp;
  const int l0 = grp * lpg, l1 = min(D.m, l0 + lpg);
  const size_t base = ((((size_t)u * D.ns + k) * ngrp + grp) * n) * n;
  if (l0 >= l1) {  // a group without modes (strips of few rows) adds zero
    for (int x = 0; x < n; ++x) {
      cst(P0 + 2 * (base + (size_t)x * n + j), cx{0.0, 0.0});
      cst(P1 + 2 * (base + (size_t)x * n + j), cx{0.0, 0.0});
    }
    return;
  }
  for (int l = l0; l < l1; ++l) {
    const double s = D.ym[2 * D.m + l];
    const double w0 = s * s, w1 = (l & 1) ? -s * s : s * s;
    const bool first = l == l0;
    auto acc = [&](int x, cx v) {
      double *p0 = P0 + 2 * (base + (size_t)x * n + j), *p1 = P1 + 2 * (base + (size_t)x * n + j);
      if (first) {
        cst(p0, cscl(v, w0));
        cst(p1, cscl(v, w1));
      } else {
        cst(p0, cadd(cld(p0), cscl(v, w0)));
        cst(p1, cadd(cld(p1), cscl(v, w1)));
      }
    };
    cx dg, of, ofm = {0.0, 0.0};
    tri_row(D, k, l, lam, j, dg, of);
    if (j > 0) {
      cx d2;
      tri_row(D, k, l, lam, j - 1, d2, ofm);
    }
    cx piv = dg;
    if (j > 0) piv = csub(piv, cmul(cmul(ofm, ofm), cld(fac_at(D, kInvD, u, k, j - 1, l))));
    if (j + 1 < n) piv = csub(piv, cmul(cmul(of, of), cld(fac_at(D, kInvB, u, k, j + 1, l))));
    const cx xj = crcp(piv);
    acc(j, xj);
    cx v = xj;
    for (int i = j - 1; i >= 0; --i) {  // above the pivot row
      cx d2, oi;
      tri_row(D, k, l, lam, i, d2, oi);
      v = cmul(cscl(cmul(oi, cld(fac_at(D, kInvD, u, k, i, l))), -1.0), v);
      acc(i, v);
    }
    v = xj;
    cx oprev = of;  // coupling (i-1, i) for i = j+1
    for (int i = j + 1; i < n; ++i) {  // below the pivot row
      v = cmul(cscl(cmul(oprev, cld(fac_at(D, kInvB, u, k, i, l))), -1.0), v);
      acc(i, v);
      cx d2;
      tri_row(D, k, l, lam, i, d2, oprev);
    }
  }
}

// G0 / G1[u][k][x][j] = sum over the groups in order (deterministic)
__global__ void k_fdm_green_sum(const FdmDesc D, int ngrp, const double *P0, const double *P1,
                                double *G0, double *G1) {
  const long long g = gid64();
  const long long nn = (long long)D.n * D.n;
  if (g >= (long long)D.nu * D.ns * nn) return;
  const long long uk = g / nn, e = g - uk * nn;
  cx a = {0.0, 0.0}, b = {0.0, 0.0};
  for (int grp = 0; grp < ngrp; ++grp) {
    const size_t o = 2 * (((size_t)uk * ngrp + grp) * nn + e);
    a = cadd(a, cld(P0 + o));
    b = cadd(b, cld(P1 + o));
  }
  cst(G0 + 2 * g, a);
  cst(G1 + 2 * g, b);
}

// (C_k A C_k)[p][q] with A the n x n block of strip k (G0 or G1)
__device__ __forceinline__ cx cac(const FdmDesc &D, int k, cx lam, const double *A, int p,
                                  int q) {
  const int n = D.n;
  cx cp[3], cq[3];
  for (int o = -1; o <= 1; ++o) {
    cx dg, of;
    cp[o + 1] = {0.0, 0.0};
    cq[o + 1] = {0.0, 0.0};
    const int pp = p + o, qq = q + o;
    if (pp >= 0 && pp < n) {
      // C[p][pp]: diagonal for o = 0, coupling (min, min+1) otherwise
      cpl_row(D, k, lam, o < 0 ? pp : p, dg, of);
      cp[o + 1] = o == 0 ? dg : of;
    }
    if (qq >= 0 && qq < n) {
      cpl_row(D, k, lam, o < 0 ? qq : q, dg, of);
      cq[o + 1] = o == 0 ? dg : of;
    }
  }
  cx r = {0.0, 0.0};
  for (int a = 0; a < 3; ++a) {
    const int pp = p + a - 1;
    if (pp < 0 || pp >= n) continue;
    cx row = {0.0, 0.0};
    for (int b = 0; b < 3; ++b) {
      const int qq = q + b - 1;
      if (qq < 0 || qq >= n) continue;
      row = cadd(row, cmul(cld(A + 2 * ((size_t)pp * n + qq)), cq[b]));
    }
    r = cadd(r, cmul(cp[a], row));
  }
  return r;
}

// The interface Schur complement, entry (rho, sigma) = ((r-1) n + p, (r'-1) n + q):
//   r' = r:      D_r - C_{r-1} G0_{r-1} C_{r-1} - C_r G0_r C_r
//   r' = r + 1:  -C_r G1_r C_r     (strip r lies between interfaces r and r+1)
//   r' = r - 1:  -C_{r-1} G1_{r-1} C_{r-1}
__global__ void k_fdm_schur(const FdmDesc D, const double *G0, const double *G1) {
  const long long g = gid64();
  const long long NG = (long long)D.ni * D.n;
  if (g >= (long long)D.nu * NG * NG) return;
  const int n = D.n;
  const long long u = g / (NG * NG), e = g - u * NG * NG;
  const int rho = (int)(e / NG), sig = (int)(e - (long long)rho * NG);
  const int r = rho / n + 1, p = rho % n, r2 = sig / n + 1, q = sig % n;
  const cx lam = cld(D.lam + 2 * u);
  const size_t nn = (size_t)n * n;
  auto blk = [&](const double *G, int k) { return G + 2 * (((size_t)u * D.ns + k) * nn); };
  cx v = {0.0, 0.0};
  if (r2 == r) {
    cx dg, of;
    if (q == p) {
      dif_row(D, r, lam, p, dg, of);
      v = dg;
    } else if (q == p + 1) {
      dif_row(D, r, lam, p, dg, of);
      v = of;
    } else if (q == p - 1) {
      dif_row(D, r, lam, q, dg, of);
      v = of;
    }
    v = csub(v, cac(D, r - 1, lam, blk(G0, r - 1), p, q));
    v = csub(v, cac(D, r, lam, blk(G0, r), p, q));
  } else if (r2 == r + 1) {
    v = cscl(cac(D, r, lam, blk(G1, r), p, q), -1.0);
  } else if (r2 == r - 1) {
    v = cscl(cac(D, r - 1, lam, blk(G1, r - 1), p, q), -1.0);
  }
  cst(D.Sinv + 2 * g, v);
}

// Gauss-Jordan inversion in place with partial pivoting, one column step.
// Pivot: one workgroup per matrix finds the pivot row, swaps it into row k
// and saves the scaled pivot row and the pivot column.
__global__ void __launch_bounds__(256) k_gj_pivot(double *S, int N, int k, double *prow,
                                                  double *fcol, int *piv) {
  const int u = blockIdx.x;
  double *A = S + 2 * (size_t)u * N * N;
  double *pr = prow + 2 * (size_t)u * N, *fc = fcol + 2 * (size_t)u * N;
  __shared__ double s_v[256];
  __shared__ int s_i[256];
  double best = -1.0;
  int bi = N;
  for (int i = k + (int)threadIdx.x; i < N; i += 256) {
    const cx a = cld(A + 2 * ((size_t)i * N + k));
    const double v = a.r * a.r + a.i * a.i;
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  s_v[threadIdx.x] = best;
  s_i[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double v2 = s_v[threadIdx.x + o];
      const int i2 = s_i[threadIdx.x + o];
      if (v2 > s_v[threadIdx.x] || (v2 == s_v[threadIdx.x] && i2 < s_i[threadIdx.x])) {
        s_v[threadIdx.x] = v2;
        s_i[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  const int p = s_i[0];
  if (p != k)
    for (int j = threadIdx.x; j < N; j += 256) {
      double *a = A + 2 * ((size_t)k * N + j), *b = A + 2 * ((size_t)p * N + j);
      const double t0 = a[0], t1 = a[1];
      a[0] = b[0];
      a[1] = b[1];
      b[0] = t0;
      b[1] = t1;
    }
  __syncthreads();
  const cx d = crcp(cld(A + 2 * ((size_t)k * N + k)));
  for (int j = threadIdx.x; j < N; j += 256) {
    cst(pr + 2 * j, j == k ? d : cmul(cld(A + 2 * ((size_t)k * N + j)), d));
    cst(fc + 2 * j, j == k ? cx{0.0, 0.0} : cld(A + 2 * ((size_t)j * N + k)));
  }
  if (threadIdx.x == 0) piv[(size_t)u * N + k] = p;
}

__global__ void k_gj_update(double *S, int N, int k, const double *prow, const double *fcol) {
  const long long e = gid64();
  if (e >= (long long)N * N) return;
  const int u = blockIdx.y;
  double *A = S + 2 * (size_t)u * N * N;
  const double *pr = prow + 2 * (size_t)u * N, *fc = fcol + 2 * (size_t)u * N;
  const int i = (int)(e / N), j = (int)(e - (long long)i * N);
  double *a = A + 2 * e;
  if (i == k)
    cst(a, cld(pr + 2 * j));
  else if (j == k)
    cst(a, cscl(cmul(cld(fc + 2 * i), cld(pr + 2 * k)), -1.0));
  else
    cst(a, csub(cld(a), cmul(cld(fc + 2 * i), cld(pr + 2 * j))));
}

// undo the row interchanges as column interchanges, last first
__global__ void k_gj_colswap(double *S, int N, const int *piv) {
  const int i = (int)gid64();
  if (i >= N) return;
  const int u = blockIdx.y;
  double *row = S + 2 * ((size_t)u * N * N + (size_t)i * N);
  const int *pv = piv + (size_t)u * N;
  for (int k = N - 1; k >= 0; --k) {
    const int p = pv[k];
    if (p == k) continue;
    const double t0 = row[2 * k], t1 = row[2 * k + 1];
    row[2 * k] = row[2 * p];
    row[2 * k + 1] = row[2 * p + 1];
    row[2 * p] = t0;
    row[2 * p + 1] = t1;
  }
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_fdm_in(const FdmDesc *d, int nd, const FdmTotals &t, hipStream_t s) {
  if (nd == 0 || t.node == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fdm_in, dim3(nblk(t.node, 256)), dim3(256), 0, s, d, nd, t.node);
  return hipGetLastError();
}

hipError_t launch_fdm_tri(const FdmDesc *d, int nd, const FdmTotals &t, int correction,
                          int chunk, hipStream_t s) {
  if (nd == 0 || t.tri == 0) return hipSuccess;
  const dim3 grid(nblk(t.tri, 64));
  if (chunk <= 4)
    hipLaunchKernelGGL(k_fdm_tri<4>, grid, dim3(64), 0, s, d, nd, t.tri, correction);
  else if (chunk <= 8)
    hipLaunchKernelGGL(k_fdm_tri<8>, grid, dim3(64), 0, s, d, nd, t.tri, correction);
  else
    hipLaunchKernelGGL(k_fdm_tri<16>, grid, dim3(64), 0, s, d, nd, t.tri, correction);
  return hipGetLastError();
}

hipError_t launch_fdm_interface(const FdmDesc *d, int nd, const FdmTotals &t, hipStream_t s) {
  if (nd == 0 || t.iface == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fdm_edge, dim3(nblk(t.edge * 16, 256)), dim3(256), 0, s, d, nd, t.edge);
  hipLaunchKernelGGL(k_fdm_iface, dim3(nblk(t.iface, 256)), dim3(256), 0, s, d, nd, t.iface);
  hipLaunchKernelGGL(k_fdm_gemv, dim3(nblk(t.gemv * 64, 256)), dim3(256), 0, s, d, nd, t.gemv);
  return hipGetLastError();
}

hipError_t launch_fdm_out(const FdmDesc *d, int nd, const FdmTotals &t, hipStream_t s) {
  if (nd == 0 || t.node == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fdm_out, dim3(nblk(t.node, 256)), dim3(256), 0, s, d, nd, t.node);
  return hipGetLastError();
}

hipError_t fdm_assemble(const FdmDesc &h) {
  hipError_t e;
  hipLaunchKernelGGL(k_fdm_factor, dim3(nblk((long long)h.nu * h.ns * h.m, 64)), dim3(64), 0,
                     nullptr, h);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (h.ni == 0) return hipDeviceSynchronize();
  const int ngrp = 8;
  const size_t nn = (size_t)h.n * h.n, blk = (size_t)h.nu * h.ns * nn;
  const int N = h.ni * h.n;
  double *P0 = nullptr, *P1 = nullptr, *G0 = nullptr, *G1 = nullptr, *prow = nullptr,
         *fcol = nullptr;
  int *piv = nullptr;
  auto cleanup = [&]() {
    for (void *q : {(void *)P0, (void *)P1, (void *)G0, (void *)G1, (void *)prow,
                    (void *)fcol, (void *)piv})
      if (q) (void)hipFree(q);
  };
  if ((e = hipMalloc(&P0, 2 * blk * ngrp * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&P1, 2 * blk * ngrp * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&G0, 2 * blk * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&G1, 2 * blk * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&prow, 2 * (size_t)h.nu * N * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&fcol, 2 * (size_t)h.nu * N * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&piv, (size_t)h.nu * N * sizeof(int))) != hipSuccess) {
    cleanup();
    return e;
  }
  hipLaunchKernelGGL(k_fdm_green, dim3(nblk((long long)h.nu * h.ns * ngrp * h.n, 64)), dim3(64),
                     0, nullptr, h, ngrp, P0, P1);
  hipLaunchKernelGGL(k_fdm_green_sum, dim3(nblk((long long)blk, 256)), dim3(256), 0, nullptr, h,
                     ngrp, P0, P1, G0, G1);
  hipLaunchKernelGGL(k_fdm_schur, dim3(nblk((long long)h.nu * N * N, 256)), dim3(256), 0,
                     nullptr, h, G0, G1);
  if ((e = hipGetLastError()) != hipSuccess) {
    cleanup();
    return e;
  }
  const dim3 ug(nblk((long long)N * N, 256), h.nu);
  for (int k = 0; k < N; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(h.nu), dim3(256), 0, nullptr, h.Sinv, N, k, prow, fcol,
                       piv);
    hipLaunchKernelGGL(k_gj_update, ug, dim3(256), 0, nullptr, h.Sinv, N, k, prow, fcol);
  }
  hipLaunchKernelGGL(k_gj_colswap, dim3(nblk(N, 256), h.nu), dim3(256), 0, nullptr, h.Sinv, N,
                     piv);
  if ((e = hipGetLastError()) == hipSuccess) e = hipDeviceSynchronize();
  cleanup();
  return e;
}

}  // namespace sg
