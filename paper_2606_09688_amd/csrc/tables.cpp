// Host-side tables of the discrete operator.  See tables.hpp.
//
// Time space (paper Sec. 2.2 and Rem. 1, p_t = 2 with C^1 continuity):
// clamped uniform knots tau = (0,0,0,h,...,(N-1)h,T,T,T), N = 2^b, basis
// B_0..B_{N+1}; B_0 is the only function nonzero at t = 0 and is dropped
// (w(0) = 0), leaving psi_i = B_{i+1}, i = 0..N.
//
// Accuracy.  Every evaluation happens in the local coordinate s in [0,1] of
// an element with knots measured in units of h from the element start (small
// integers), so no cancellation t - tau occurs.  On element e the three
// nonzero B-splines are exact quadratics in s; with t = T (e+s)/N the weight
// is e^{-t/T} = e^{-e/N} e^{-s/N}, and every integral is a combination of the
// moments I_k = int_0^1 s^k e^{-s/N} ds, evaluated by their series in
// double-double.  The time matrices A_b, B_b are kept as double-double
// (hi + lo): the discrete solution of long time levels is sensitive to
// last-bit perturbations of their entries, and the solver's refinement uses
// the exact entries.  Everything else is rounded once to double.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <stdexcept>

#include "dd.hpp"

namespace sg {

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) /
                         (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        long double pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    x[i] = (double)z;
    w[i] = (double)(2 / ((1 - z * z) * dp * dp));
  }
}

// knot tau_k of the clamped uniform knot vector with N intervals, in units of h
static int ref_knot(int N, int k) {
  if (k <= 2) return 0;
  if (k >= N + 2) return N;
  return k - 2;
}

// Values / derivatives (in units of 1/h, 1/h^2) of B_e, B_{e+1}, B_{e+2} at
// the local coordinate s of element e, knots relative to the element start.
static void spline_ref(int N, int e, double s, double v[3], double d1[3], double d2[3]) {
  const int sp = e + 2;  // knot span
  const double tm1 = ref_knot(N, sp - 1) - e, t0 = ref_knot(N, sp) - e,
               t1 = ref_knot(N, sp + 1) - e, t2 = ref_knot(N, sp + 2) - e;
  const double dl = t1 - t0, da = t1 - tm1, db = t2 - t0;
  const double n0 = (t1 - s) / dl, n1 = (s - t0) / dl;
  v[0] = (t1 - s) / da * n0;
  v[1] = (s - tm1) / da * n0 + (t2 - s) / db * n1;
  v[2] = (s - t0) / db * n1;
  d1[0] = -2.0 * n0 / da;
  d1[1] = 2.0 * (n0 / da - n1 / db);
  d1[2] = 2.0 * n1 / db;
  d2[0] = 2.0 / (dl * da);
  d2[1] = -2.0 / dl * (1.0 / da + 1.0 / db);
  d2[2] = 2.0 / (dl * db);
}

// Exact quadratic coefficients c[f][k] (B_{e+f}(s) = sum_k c[f][k] s^k).
static void local_poly(int N, int e, double c[3][3]) {
  double v0[3], v5[3], v1[3], d1[3], d2[3];
  spline_ref(N, e, 0.0, v0, d1, d2);
  spline_ref(N, e, 0.5, v5, d1, d2);
  spline_ref(N, e, 1.0, v1, d1, d2);
  for (int f = 0; f < 3; ++f) {
    c[f][0] = v0[f];
    c[f][2] = 2.0 * (v1[f] - 2.0 * v5[f] + v0[f]);
    c[f][1] = v1[f] - v0[f] - c[f][2];
  }
}

void spline_local(int b, double T, int e, double t, double v[3], double d1[3],
                  double d2[3]) {
  const int N = 1 << b;
  const double h = T / N;
  spline_ref(N, e, t / h - e, v, d1, d2);
  for (int f = 0; f < 3; ++f) {
    d1[f] /= h;
    d2[f] /= h * h;
  }
}

TimeLevel time_level(int b, double T) {
  TimeLevel L;
  const int N = 1 << b;
  L.b = b;
  L.nq = N + 1;
  const ddv lam(1.0 / N);
  ddv I[5];
  for (int k = 0; k < 5; ++k) I[k] = moment(k, lam);
  const ddv E1 = exp_neg(lam);
  std::vector<ddv> Ar((size_t)L.nq * 5), Br((size_t)L.nq * 5), gr(L.nq);
  ddv Ee(1.0);  // e^{-e/N}
  for (int e = 0; e < N; ++e) {
    double c[3][3];
    local_poly(N, e, c);
    for (int fi = 0; fi < 3; ++fi) {
      const int i = e + fi - 1;  // B_{e+fi} = psi_{e+fi-1}
      if (i < 0) continue;
      const double di0 = c[fi][1], di1 = 2.0 * c[fi][2];  // B' = di0 + di1 s
      const ddv gi = ddv(di0) * I[0] + ddv(di1) * I[1];
      gr[i] += Ee * gi;
      for (int fj = 0; fj < 3; ++fj) {
        const int j = e + fj - 1;
        if (j < 0) continue;
        const double dd2 = 2.0 * c[fj][2];  // B''
        const ddv a = ddv(dd2) * gi;
        ddv bb(0.0);
        for (int k = 0; k < 3; ++k)
          bb += ddv(c[fj][k]) * (ddv(di0) * I[k] + ddv(di1) * I[k + 1]);
        Ar[(size_t)i * 5 + (j - i + 2)] += Ee * a;
        Br[(size_t)i * 5 + (j - i + 2)] += Ee * bb;
      }
    }
    Ee = Ee * E1;
  }
  // penalty psi_j'(0) psi_i'(0): only psi_0 = B_1 has a slope at 0 (2/h)
  Ar[2] += ddv(4.0);
  const ddv NT = ddv((double)N) / ddv(T);
  const ddv sc = NT * NT;  // A scales as (N/T)^2; B and g do not depend on T
  L.A.assign((size_t)L.nq * 5, 0.0);
  L.Alo.assign((size_t)L.nq * 5, 0.0);
  L.B.assign((size_t)L.nq * 5, 0.0);
  L.Blo.assign((size_t)L.nq * 5, 0.0);
  for (size_t k = 0; k < Ar.size(); ++k) {
    const ddv a = sc * Ar[k];
    L.A[k] = a.hi;
    L.Alo[k] = a.lo;
    L.B[k] = Br[k].hi;
    L.Blo[k] = Br[k].lo;
  }
  L.g.resize(L.nq);
  for (int i = 0; i < L.nq; ++i) L.g[i] = gr[i].value();
  const double nt = NT.value();
  L.d0 = 2.0 * nt;
  // psi_i'(t_i) and psi_i'(t_{i+1}) from the local slopes at element ends
  L.Dlo.assign(L.nq, 0.0);
  L.Dhi.assign(L.nq, 0.0);
  double v[3], d1[3], d2[3];
  for (int i = 0; i <= N; ++i) {
    for (int side = 0; side < 2; ++side) {
      const int q = i + side;
      if (q > N) continue;
      const int e = q < N ? q : N - 1;
      spline_ref(N, e, q < N ? 0.0 : 1.0, v, d1, d2);
      const int f = (i + 1) - e;
      const double val = (f >= 0 && f <= 2) ? d1[f] * nt : 0.0;
      (side == 0 ? L.Dlo : L.Dhi)[i] = val;
    }
  }
  return L;
}

static void normalise_taps(int nq, int n, int qmin, const double *vals, int nv,
                           Taps &tp) {
  int q0 = qmin;
  if (q0 > nq - 3) q0 = nq - 3;
  if (q0 < 0) q0 = 0;
  tp.q0[n] = q0;
  for (int k = 0; k < 3; ++k) tp.w[3 * (size_t)n + k] = 0.0;
  for (int k = 0; k < nv; ++k) {
    const int slot = qmin + k - q0;
    if (vals[k] == 0.0) continue;
    if (slot < 0 || slot > 2) throw std::runtime_error("tap outside window");
    tp.w[3 * (size_t)n + slot] = vals[k];
  }
}

Taps p1_taps(int b, int J, double T) {
  const int N = 1 << J, nq = (1 << b) + 1, s = 1 << (J - b);
  // fine weighted P1 mass on element n: (T/N) e^{-n/N} int phi_a phi_b e^{-s/N}
  const ddv lam(1.0 / N);
  const ddv I0 = moment(0, lam), I1 = moment(1, lam), I2 = moment(2, lam);
  const ddv m00 = I0 - ddv(2.0) * I1 + I2, m01 = I1 - I2, m11 = I2;
  const ddv E1 = exp_neg(lam), hT = ddv(T) / ddv((double)N);
  std::vector<ddv> md(N + 1), mo(N);
  ddv Ee(1.0);
  for (int e = 0; e < N; ++e) {
    const ddv f = hT * Ee;
    md[e] += f * m00;
    md[e + 1] += f * m11;
    mo[e] = f * m01;
    Ee = Ee * E1;
  }
  auto lam_q = [&](int q, int n) {  // P1 hat of level-b node q at fine node n
    const int dist = n > q * s ? n - q * s : q * s - n;
    return dist >= s ? 0.0 : 1.0 - (double)dist / s;
  };
  Taps tp;
  tp.q0.assign(N + 1, 0);
  tp.w.assign(3 * (size_t)(N + 1), 0.0);
  for (int n = 0; n <= N; ++n) {
    double vals[8] = {0};
    int qmin = -1, nv = 0;
    const int qa = (n - 1 - s) / s - 1, qz = (n + 1 + s) / s + 1;
    for (int q = qa < 0 ? 0 : qa; q <= qz && q < nq; ++q) {
      ddv acc = ddv(lam_q(q, n)) * md[n];
      if (n > 0) acc += ddv(lam_q(q, n - 1)) * mo[n - 1];
      if (n < N) acc += ddv(lam_q(q, n + 1)) * mo[n];
      if (acc.hi != 0.0) {
        if (qmin < 0) qmin = q;
        vals[q - qmin] = acc.value();
        nv = q - qmin + 1;
      }
    }
    if (nv > 3) throw std::runtime_error("P1 taps wider than 3");
    normalise_taps(nq, n, qmin, vals, nv, tp);
  }
  return tp;
}

Taps spline_taps(int b, int J, double T) {
  (void)T;
  const int N = 1 << J, nb = 1 << b, s = 1 << (J - b);
  Taps tp;
  tp.q0.assign(N + 1, 0);
  tp.w.assign(3 * (size_t)(N + 1), 0.0);
  double v[3], d1[3], d2[3];
  for (int n = 0; n <= N; ++n) {
    int e = n / s;
    if (e > nb - 1) e = nb - 1;
    spline_ref(nb, e, (double)(n - e * s) / s, v, d1, d2);
    // B_{e+k} is psi_{e+k-1}; B_0 (k=0 when e=0) is not in the space
    double vals[3];
    int qmin = e - 1, nv = 3;
    for (int k = 0; k < 3; ++k) vals[k] = v[k];
    if (e == 0) {
      vals[0] = v[1];
      vals[1] = v[2];
      qmin = 0;
      nv = 2;
    }
    normalise_taps(nb + 1, n, qmin, vals, nv, tp);
  }
  return tp;
}

Taps spline_taps_at(int b, double T, const std::vector<double> &t, int deriv) {
  const int nb = 1 << b;
  const double h = T / nb;
  Taps tp;
  tp.q0.assign(t.size(), 0);
  tp.w.assign(3 * t.size(), 0.0);
  double v[3], d1[3], d2[3];
  for (size_t n = 0; n < t.size(); ++n) {
    int e = (int)std::floor(t[n] / h);
    if (e < 0) e = 0;
    if (e > nb - 1) e = nb - 1;
    spline_ref(nb, e, t[n] / h - e, v, d1, d2);
    double vals[3];
    for (int k = 0; k < 3; ++k) vals[k] = deriv ? d1[k] / h : v[k];
    // B_{e+k} is psi_{e+k-1}; B_0 (k = 0 on element 0) is not in the space
    int qmin = e - 1, nv = 3;
    if (e == 0) {
      vals[0] = vals[1];
      vals[1] = vals[2];
      qmin = 0;
      nv = 2;
    }
    normalise_taps(nb + 1, (int)n, qmin, vals, nv, tp);
  }
  return tp;
}

Taps sum_taps(int J) {
  const int N = 1 << J;
  Taps tp;
  tp.q0.assign(N + 1, 0);
  tp.w.assign(3 * (size_t)(N + 1), 0.0);
  for (int n = 0; n <= N; ++n) tp.w[3 * (size_t)n] = 1.0;
  return tp;
}

void p1_eigen(int a, double len, std::vector<double> &m, std::vector<double> &k) {
  const int n = 1 << a;
  const long double h = (long double)len / n;
  const long double pi = 3.14159265358979323846264338327950288L;
  m.resize(n - 1);
  k.resize(n - 1);
  for (int j = 1; j < n; ++j) {
    const long double th = pi * j / n;
    const long double sh = sinl(th / 2);
    m[j - 1] = (double)(h / 6 * (4 + 2 * cosl(th)));
    k[j - 1] = (double)(4 / h * sh * sh);
  }
}

std::vector<double> dst_matrix(int a) {
  const int n = 1 << a, m = n - 1;
  const long double pi = 3.14159265358979323846264338327950288L;
  const long double sc = sqrtl(2.0L / n);
  std::vector<double> Q((size_t)m * m);
  for (int j = 1; j < n; ++j)
    for (int k = 1; k < n; ++k) {
      const long long r = ((long long)j * k) % (2 * n);  // sin(pi r / n)
      Q[(size_t)(j - 1) * m + (k - 1)] = (double)(sc * sinl(pi * r / n));
    }
  return Q;
}

}  // namespace sg

namespace sg {

// ---------------------------------------------------------------------------
// Variable wave speed, d = 1.

std::vector<double> element_c2(int a, double len, int ncell, const double *c_vals) {
  const int ne = 1 << a;
  std::vector<double> out(ne, 0.0);
  // element e = [e, e+1] * len / ne, block b = [b, b+1] * len / ncell; the
  // overlap in units of len / (ne * ncell) is an integer count
  for (int e = 0; e < ne; ++e) {
    const long long lo = (long long)e * ncell, hi = lo + ncell;  // element in fine units
    long double acc = 0.0L;
    for (int b = 0; b < ncell; ++b) {
      const long long blo = (long long)b * ne, bhi = blo + ne;
      const long long ov = std::min(hi, bhi) - std::max(lo, blo);
      if (ov > 0) acc += (long double)c_vals[b] * c_vals[b] * ov;
    }
    out[e] = (double)(acc / ncell);
  }
  return out;
}

// Symmetric eigen-decomposition by the cyclic Jacobi method: on return C is
// (numerically) diagonal and Q (row-major, columns = eigenvectors) satisfies
// C_in = Q diag(C) Q^T.
static void jacobi_eigen(int n, std::vector<long double> &C, std::vector<long double> &Q) {
  Q.assign((size_t)n * n, 0.0L);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0L;
  auto c = [&](int i, int j) -> long double & { return C[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    long double off = 0.0L, diag = 0.0L;
    for (int i = 0; i < n; ++i) {
      diag += c(i, i) * c(i, i);
      for (int j = i + 1; j < n; ++j) off += c(i, j) * c(i, j);
    }
    if (off <= 1e-38L * diag) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const long double apq = c(p, q);
        if (apq == 0.0L) continue;
        const long double theta = (c(q, q) - c(p, p)) / (2.0L * apq);
        const long double t = (theta >= 0 ? 1.0L : -1.0L) /
                              (fabsl(theta) + sqrtl(theta * theta + 1.0L));
        const long double cs = 1.0L / sqrtl(t * t + 1.0L), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const long double kp = c(k, p), kq = c(k, q);
          c(k, p) = cs * kp - sn * kq;
          c(k, q) = sn * kp + cs * kq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const long double pk = c(p, k), qk = c(q, k);
          c(p, k) = cs * pk - sn * qk;
          c(q, k) = sn * pk + cs * qk;
        }
        c(p, q) = c(q, p) = 0.0L;
        for (int k = 0; k < n; ++k) {
          long double &kp = Q[(size_t)k * n + p], &kq = Q[(size_t)k * n + q];
          const long double a0 = kp, a1 = kq;
          kp = cs * a0 - sn * a1;
          kq = sn * a0 + cs * a1;
        }
      }
  }
}

void pencil_eigen(int a, double len, const std::vector<double> &c2e, std::vector<double> &V,
                  std::vector<double> &lam) {
  const int ne = 1 << a, n = ne - 1;
  const long double h = (long double)len / ne;
  // M = h/6 tridiag(1,4,1); K[i][i] = (c2_{i} + c2_{i+1})/h, K[i][i+1] = -c2_{i+1}/h
  // (interior node i+1 sits between elements i and i+1)
  std::vector<long double> md(n, 4.0L * h / 6.0L), mo(n, h / 6.0L);
  std::vector<long double> kd(n), ko(n, 0.0L);
  for (int i = 0; i < n; ++i) {
    kd[i] = (c2e[i] + c2e[i + 1]) / h;
    if (i + 1 < n) ko[i] = -(long double)c2e[i + 1] / h;
  }
  // M = L L^T, L lower bidiagonal (diagonal ld, subdiagonal ls)
  std::vector<long double> ld(n), ls(n, 0.0L);
  for (int i = 0; i < n; ++i) {
    const long double d = md[i] - (i > 0 ? ls[i - 1] * ls[i - 1] : 0.0L);
    ld[i] = sqrtl(d);
    if (i + 1 < n) ls[i] = mo[i] / ld[i];
  }
  // C = L^{-1} K L^{-T}: X = L^{-1} K (columns), C = L^{-1} X^T, symmetrised
  std::vector<long double> X((size_t)n * n, 0.0L), C((size_t)n * n, 0.0L);
  for (int j = 0; j < n; ++j) {
    long double prev = 0.0L;
    for (int i = 0; i < n; ++i) {
      long double kij = 0.0L;
      if (i == j) kij = kd[i];
      else if (i == j + 1) kij = ko[j];
      else if (j == i + 1) kij = ko[i];
      const long double x = (kij - (i > 0 ? ls[i - 1] * prev : 0.0L)) / ld[i];
      X[(size_t)i * n + j] = x;
      prev = x;
    }
  }
  for (int j = 0; j < n; ++j) {  // column j of C = L^{-1} (row j of X)
    long double prev = 0.0L;
    for (int i = 0; i < n; ++i) {
      const long double x = (X[(size_t)j * n + i] - (i > 0 ? ls[i - 1] * prev : 0.0L)) / ld[i];
      C[(size_t)i * n + j] = x;
      prev = x;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const long double s = 0.5L * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
      C[(size_t)i * n + j] = C[(size_t)j * n + i] = s;
    }
  std::vector<long double> Q;
  jacobi_eigen(n, C, Q);
  lam.resize(n);
  for (int k = 0; k < n; ++k) lam[k] = (double)C[(size_t)k * n + k];
  // V = L^{-T} Q (back substitution per column); V^T M V = I
  V.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    long double next = 0.0L;
    for (int i = n - 1; i >= 0; --i) {
      const long double v = (Q[(size_t)i * n + k] - (i + 1 < n ? ls[i] * next : 0.0L)) / ld[i];
      V[(size_t)i * n + k] = (double)v;
      next = v;
    }
  }
}

}  // namespace sg

namespace sg {

// Block LU of S = A (x) M + B (x) K in space-major order (see tables.hpp).
void block_lu(const TimeLevel &tl, const std::vector<double> &mk, int nx,
              std::vector<double> &Dinv, std::vector<double> &Lf) {
  const int nq = tl.nq;
  typedef long double R;
  auto band = [&](const std::vector<double> &hi, const std::vector<double> &lo, int i,
                  int j) -> R {
    const int off = j - i;
    if (off < -2 || off > 2) return 0.0L;
    return (R)hi[(size_t)i * 5 + off + 2] + (R)lo[(size_t)i * 5 + off + 2];
  };
  std::vector<R> Ad((size_t)nq * nq), Bd((size_t)nq * nq);
  for (int i = 0; i < nq; ++i)
    for (int j = 0; j < nq; ++j) {
      Ad[(size_t)i * nq + j] = band(tl.A, tl.Alo, i, j);
      Bd[(size_t)i * nq + j] = band(tl.B, tl.Blo, i, j);
    }
  auto blockS = [&](R m, R k, std::vector<R> &S) {
    for (size_t e = 0; e < S.size(); ++e) S[e] = m * Ad[e] + k * Bd[e];
  };
  // inverse by Gauss-Jordan elimination with partial pivoting
  auto invert = [&](std::vector<R> D, std::vector<R> &Inv) {
    Inv.assign((size_t)nq * nq, 0.0L);
    for (int i = 0; i < nq; ++i) Inv[(size_t)i * nq + i] = 1.0L;
    for (int c = 0; c < nq; ++c) {
      int piv = c;
      for (int r = c + 1; r < nq; ++r)
        if (fabsl(D[(size_t)r * nq + c]) > fabsl(D[(size_t)piv * nq + c])) piv = r;
      if (piv != c)
        for (int j = 0; j < nq; ++j) {
          std::swap(D[(size_t)c * nq + j], D[(size_t)piv * nq + j]);
          std::swap(Inv[(size_t)c * nq + j], Inv[(size_t)piv * nq + j]);
        }
      const R d = D[(size_t)c * nq + c];
      for (int j = 0; j < nq; ++j) {
        D[(size_t)c * nq + j] /= d;
        Inv[(size_t)c * nq + j] /= d;
      }
      for (int r = 0; r < nq; ++r) {
        if (r == c) continue;
        const R f = D[(size_t)r * nq + c];
        if (f == 0.0L) continue;
        for (int j = 0; j < nq; ++j) {
          D[(size_t)r * nq + j] -= f * D[(size_t)c * nq + j];
          Inv[(size_t)r * nq + j] -= f * Inv[(size_t)c * nq + j];
        }
      }
    }
  };
  const size_t bs = (size_t)nq * nq;
  Dinv.assign(bs * nx, 0.0);
  Lf.assign(bs * nx, 0.0);
  std::vector<R> D(bs), Di(bs), Soff(bs), Lk(bs), tmp(bs);
  // K entries as hi + lo (extended precision)
  auto kk = [&](int k, int o) -> R { return (R)mk[kSpaceStride * k + 2 + o] + (R)mk[kSpaceStride * k + 4 + o]; };
  blockS(mk[0], kk(0, 0), D);
  invert(D, Di);
  for (size_t e = 0; e < bs; ++e) Dinv[e] = (double)Di[e];
  for (int k = 1; k < nx; ++k) {
    // S_{k,k-1} = S_{k-1,k} (M and K symmetric)
    blockS(mk[kSpaceStride * (k - 1) + 1], kk(k - 1, 1), Soff);
    for (int i = 0; i < nq; ++i)
      for (int j = 0; j < nq; ++j) {
        R acc = 0.0L;
        for (int l = 0; l < nq; ++l) acc += Soff[(size_t)i * nq + l] * Di[(size_t)l * nq + j];
        Lk[(size_t)i * nq + j] = acc;
      }
    blockS(mk[kSpaceStride * k], kk(k, 0), D);
    for (int i = 0; i < nq; ++i)
      for (int j = 0; j < nq; ++j) {
        R acc = 0.0L;
        for (int l = 0; l < nq; ++l) acc += Lk[(size_t)i * nq + l] * Soff[(size_t)l * nq + j];
        D[(size_t)i * nq + j] -= acc;
      }
    invert(D, Di);
    for (size_t e = 0; e < bs; ++e) {
      Dinv[bs * k + e] = (double)Di[e];
      Lf[bs * k + e] = (double)Lk[e];
    }
  }
}

// 1-D P1 integrals of level a over [lo, hi] (part of (0, len)), per interior
// node k: mass and unit stiffness on the diagonal (d) and the coupling of
// k and k+1 (o).  On element e the hats are 1 - u and u, u = x / h - e.
struct P1Band {
  std::vector<long double> md, mo, kd, ko;
};
static P1Band p1_on_interval(int a, double len, long double lo, long double hi) {
  const int ne = 1 << a, n = ne - 1;
  const long double h = (long double)len / ne;
  P1Band B;
  B.md.assign(n, 0.0L); B.mo.assign(n, 0.0L); B.kd.assign(n, 0.0L); B.ko.assign(n, 0.0L);
  for (int e = 0; e < ne; ++e) {
    const long double x0 = std::max(lo, e * h), x1 = std::min(hi, (e + 1) * h);
    if (x1 <= x0) continue;
    const long double u0 = x0 / h - e, u1 = x1 / h - e;
    const long double d1 = u1 - u0, d2 = u1 * u1 - u0 * u0, d3 = u1 * u1 * u1 - u0 * u0 * u0;
    const long double mll = h * (d1 - d2 + d3 / 3), mlr = h * (d2 / 2 - d3 / 3), mrr = h * d3 / 3;
    const long double kk = d1 / h;
    if (e >= 1) { B.md[e - 1] += mll; B.kd[e - 1] += kk; }        // left node e
    if (e + 1 <= n) { B.md[e] += mrr; B.kd[e] += kk; }            // right node e+1
    if (e >= 1 && e + 1 <= n) { B.mo[e - 1] += mlr; B.ko[e - 1] -= kk; }
  }
  return B;
}

std::vector<double> strip_x_tables(int a, double len, int ncell, const double *c_row) {
  const int n = (1 << a) - 1;
  std::vector<long double> kd(n, 0.0L), ko(n, 0.0L), md(n, 0.0L), mo(n, 0.0L);
  for (int bx = 0; bx < ncell; ++bx) {
    const long double lo = (long double)len * bx / ncell, hi = (long double)len * (bx + 1) / ncell;
    const P1Band B = p1_on_interval(a, len, lo, hi);
    const long double c2 = (long double)c_row[bx] * c_row[bx];
    for (int k = 0; k < n; ++k) {
      kd[k] += c2 * B.kd[k];
      ko[k] += c2 * B.ko[k];
      md[k] += c2 * B.md[k];
      mo[k] += c2 * B.mo[k];
    }
  }
  std::vector<double> out(4 * (size_t)n);
  for (int k = 0; k < n; ++k) {
    out[k] = (double)kd[k];
    out[n + k] = (double)ko[k];
    out[2 * n + k] = (double)md[k];
    out[3 * n + k] = (double)mo[k];
  }
  return out;
}

void pencil_2d(int a, const double *len, const int *ncell, const double *c_vals,
               std::vector<double> &K, std::vector<double> &M) {
  const int n = (1 << a) - 1;
  const size_t n2 = (size_t)n * n;
  auto band = [](const std::vector<long double> &d, const std::vector<long double> &o, int i,
                 int j) -> long double {
    if (i == j) return d[i];
    if (j == i + 1) return o[i];
    if (i == j + 1) return o[j];
    return 0.0L;
  };
  std::vector<P1Band> bx(ncell[0]), by(ncell[1]);
  for (int b = 0; b < ncell[0]; ++b)
    bx[b] = p1_on_interval(a, len[0], (long double)len[0] * b / ncell[0],
                           (long double)len[0] * (b + 1) / ncell[0]);
  for (int b = 0; b < ncell[1]; ++b)
    by[b] = p1_on_interval(a, len[1], (long double)len[1] * b / ncell[1],
                           (long double)len[1] * (b + 1) / ncell[1]);
  const P1Band fx = p1_on_interval(a, len[0], 0.0L, len[0]);
  const P1Band fy = p1_on_interval(a, len[1], 0.0L, len[1]);
  K.assign(n2 * n2, 0.0);
  M.assign(n2 * n2, 0.0);
  for (int iy = 0; iy < n; ++iy)
    for (int ix = 0; ix < n; ++ix)
      for (int jy = std::max(0, iy - 1); jy <= std::min(n - 1, iy + 1); ++jy)
        for (int jx = std::max(0, ix - 1); jx <= std::min(n - 1, ix + 1); ++jx) {
          long double k = 0.0L;
          for (int cy = 0; cy < ncell[1]; ++cy)
            for (int cx = 0; cx < ncell[0]; ++cx) {
              const long double c = c_vals[(size_t)cy * ncell[0] + cx];
              k += c * c * (band(by[cy].md, by[cy].mo, iy, jy) * band(bx[cx].kd, bx[cx].ko, ix, jx) +
                            band(by[cy].kd, by[cy].ko, iy, jy) * band(bx[cx].md, bx[cx].mo, ix, jx));
            }
          const size_t r = (size_t)iy * n + ix, c = (size_t)jy * n + jx;
          K[r * n2 + c] = (double)k;
          M[r * n2 + c] = (double)(band(fy.md, fy.mo, iy, jy) * band(fx.md, fx.mo, ix, jx));
        }
}

std::vector<double> space_entries(int a, double len, int ncell, const double *c_vals) {
  const int ne = 1 << a, n = ne - 1;
  const double h = len / ne;  // exact: len scaled by a power of two
  // C[e] = average of c^2 over element e, in double-double: the overlap of
  // element e and block b in units of len / (ne * ncell) is an integer
  std::vector<ddv> C(ne);
  for (int e = 0; e < ne; ++e) {
    const long long lo = (long long)e * ncell, hi = lo + ncell;
    ddv acc(0.0);
    for (int b = 0; b < ncell; ++b) {
      const long long blo = (long long)b * ne, bhi = blo + ne;
      const long long ov = std::min(hi, bhi) - std::max(lo, blo);
      if (ov > 0) acc += two_prod(c_vals[b], c_vals[b]) * ddv((double)ov);
    }
    C[e] = acc / ddv((double)ncell);
  }
  std::vector<double> mk((size_t)kSpaceStride * n, 0.0);
  for (int k = 0; k < n; ++k) {
    double *r = &mk[(size_t)kSpaceStride * k];
    r[0] = 4.0 * h / 6.0;
    const ddv kd = (C[k] + C[k + 1]) / ddv(h);
    r[2] = kd.hi;
    r[4] = kd.lo;
    if (k + 1 < n) {
      r[1] = h / 6.0;
      const ddv ko = -(C[k + 1] / ddv(h));
      r[3] = ko.hi;
      r[5] = ko.lo;
    }
  }
  return mk;
}

}  // namespace sg

// ---------------------------------------------------------------------------
// Time-direction diagonalisation of a short time level (2-D variable speed).
// ---------------------------------------------------------------------------
namespace sg {

namespace {

typedef long double R;
typedef std::complex<long double> C;

// Eigenvalues of a complex upper Hessenberg matrix H (n x n, row-major) by
// the shifted QR iteration with Wilkinson shifts (Givens rotations on the
// active block, deflation at negligible subdiagonal entries).
bool hessenberg_eigenvalues(int n, std::vector<C> H, std::vector<C> &ev) {
  ev.assign(n, C(0));
  const R eps = std::numeric_limits<R>::epsilon();
  int hi = n - 1, iter = 0;
  std::vector<C> cs(n), sn(n);
  while (hi >= 0) {
    if (hi == 0) {
      ev[0] = H[0];
      break;
    }
    int lo = hi;
    while (lo > 0 && std::abs(H[(size_t)lo * n + lo - 1]) >
                         eps * (std::abs(H[(size_t)lo * n + lo]) +
                                std::abs(H[(size_t)(lo - 1) * n + lo - 1])))
      --lo;
    if (lo == hi) {
      ev[hi] = H[(size_t)hi * n + hi];
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 200) return false;
    // Wilkinson shift: eigenvalue of the trailing 2 x 2 block nearer to its
    // last diagonal entry (an exceptional shift every 11 iterations)
    const C a = H[(size_t)(hi - 1) * n + hi - 1], b = H[(size_t)(hi - 1) * n + hi];
    const C c = H[(size_t)hi * n + hi - 1], d = H[(size_t)hi * n + hi];
    C shift;
    if (iter % 11 == 0) {
      shift = d + C(std::abs(c), 0);
    } else {
      const C tr2 = (a + d) / (R)2, disc = std::sqrt(tr2 * tr2 - (a * d - b * c));
      const C m1 = tr2 + disc, m2 = tr2 - disc;
      shift = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    for (int k = lo; k <= hi; ++k) H[(size_t)k * n + k] -= shift;
    // H - shift = Q R: rotations from the left zero the subdiagonal
    for (int k = lo; k < hi; ++k) {
      const C x = H[(size_t)k * n + k], y = H[(size_t)(k + 1) * n + k];
      const R r = std::sqrt(std::norm(x) + std::norm(y));
      cs[k] = r > 0 ? x / r : C(1);
      sn[k] = r > 0 ? y / r : C(0);
      for (int j = k; j <= hi; ++j) {
        const C u = H[(size_t)k * n + j], v = H[(size_t)(k + 1) * n + j];
        H[(size_t)k * n + j] = std::conj(cs[k]) * u + std::conj(sn[k]) * v;
        H[(size_t)(k + 1) * n + j] = -sn[k] * u + cs[k] * v;
      }
    }
    // R Q + shift (rotations from the right keep the Hessenberg form)
    for (int k = lo; k < hi; ++k)
      for (int i = lo; i <= std::min(k + 1, hi); ++i) {
        const C u = H[(size_t)i * n + k], v = H[(size_t)i * n + k + 1];
        H[(size_t)i * n + k] = u * cs[k] + v * sn[k];
        H[(size_t)i * n + k + 1] = -u * std::conj(sn[k]) + v * std::conj(cs[k]);
      }
    for (int k = lo; k <= hi; ++k) H[(size_t)k * n + k] += shift;
  }
  return true;
}

// Reduction of a real matrix to upper Hessenberg form by Householder
// reflections (similarity transform; eigenvalues preserved).
std::vector<C> to_hessenberg(int n, std::vector<R> G) {
  for (int k = 0; k + 2 < n; ++k) {
    R alpha = 0;
    for (int i = k + 1; i < n; ++i) alpha += G[(size_t)i * n + k] * G[(size_t)i * n + k];
    alpha = std::sqrt(alpha);
    if (alpha == 0) continue;
    if (G[(size_t)(k + 1) * n + k] > 0) alpha = -alpha;
    std::vector<R> v(n, 0);
    v[k + 1] = G[(size_t)(k + 1) * n + k] - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = G[(size_t)i * n + k];
    R vv = 0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0) continue;
    // G = (I - 2 v v^T / vv) G (I - 2 v v^T / vv)
    for (int j = 0; j < n; ++j) {
      R s = 0;
      for (int i = k + 1; i < n; ++i) s += v[i] * G[(size_t)i * n + j];
      s *= 2 / vv;
      for (int i = k + 1; i < n; ++i) G[(size_t)i * n + j] -= s * v[i];
    }
    for (int i = 0; i < n; ++i) {
      R s = 0;
      for (int j = k + 1; j < n; ++j) s += G[(size_t)i * n + j] * v[j];
      s *= 2 / vv;
      for (int j = k + 1; j < n; ++j) G[(size_t)i * n + j] -= s * v[j];
    }
  }
  std::vector<C> H((size_t)n * n);
  for (size_t e = 0; e < H.size(); ++e) H[e] = C(G[e], 0);
  return H;
}

// Solve M x = b in place (complex, Gaussian elimination with partial
// pivoting); returns false on a zero pivot.
bool complex_solve(int n, std::vector<C> M, std::vector<C> &b) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(M[(size_t)r * n + c]) > std::abs(M[(size_t)piv * n + c])) piv = r;
    if (std::abs(M[(size_t)piv * n + c]) == 0) return false;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)c * n + j], M[(size_t)piv * n + j]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const C f = M[(size_t)r * n + c] / M[(size_t)c * n + c];
      if (f == C(0)) continue;
      for (int j = c; j < n; ++j) M[(size_t)r * n + j] -= f * M[(size_t)c * n + j];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    C s = b[r];
    for (int j = r + 1; j < n; ++j) s -= M[(size_t)r * n + j] * b[j];
    b[r] = s / M[(size_t)r * n + r];
  }
  return true;
}

}  // namespace

bool time_fdm(const TimeLevel &tl, TimeFdm &out) {
  const int n = tl.nq;
  // A and B to ~32 digits (hi + lo), then G = B^{-1} A column by column
  std::vector<R> A((size_t)n * n, 0), B((size_t)n * n, 0);
  for (int i = 0; i < n; ++i)
    for (int o = -2; o <= 2; ++o) {
      const int j = i + o;
      if (j < 0 || j >= n) continue;
      A[(size_t)i * n + j] = (R)tl.A[(size_t)i * 5 + o + 2] + (R)tl.Alo[(size_t)i * 5 + o + 2];
      B[(size_t)i * n + j] = (R)tl.B[(size_t)i * 5 + o + 2] + (R)tl.Blo[(size_t)i * 5 + o + 2];
    }
  std::vector<C> Bc((size_t)n * n);
  for (size_t e = 0; e < Bc.size(); ++e) Bc[e] = C(B[e], 0);
  std::vector<R> G((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    std::vector<C> col(n);
    for (int i = 0; i < n; ++i) col[i] = C(A[(size_t)i * n + j], 0);
    if (!complex_solve(n, Bc, col)) return false;
    for (int i = 0; i < n; ++i) G[(size_t)i * n + j] = col[i].real();
  }
  std::vector<C> ev;
  if (!hessenberg_eigenvalues(n, to_hessenberg(n, G), ev)) return false;
  // unique eigenvalues: the real ones and one of each conjugate pair (Im > 0)
  const R tol = 1e-12L;
  std::vector<C> uniq;
  std::vector<int> pair;  // 1: stands for a conjugate pair
  for (const C &l : ev) {
    if (std::abs(l.imag()) <= tol * std::abs(l)) {
      uniq.push_back(C(l.real(), 0));
      pair.push_back(0);
    } else if (l.imag() > 0) {
      uniq.push_back(l);
      pair.push_back(1);
    }
  }
  int total = 0;
  for (int p : pair) total += p ? 2 : 1;
  if (total != n) return false;  // unpaired complex eigenvalue
  // eigenvectors by inverse iteration on (G - lambda I), columns of V for
  // the full spectrum (the partner of a pair is the conjugate vector)
  std::vector<C> V((size_t)n * n);
  std::vector<int> vcol(uniq.size());
  int col = 0;
  for (size_t u = 0; u < uniq.size(); ++u) {
    const C l = uniq[u];
    std::vector<C> M((size_t)n * n);
    const R pert = 64 * std::numeric_limits<R>::epsilon() * (std::abs(l) + 1);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        M[(size_t)i * n + j] = C(G[(size_t)i * n + j], 0) - (i == j ? l + C(pert, 0) : C(0));
    std::vector<C> v(n, C(1));
    for (int it = 0; it < 3; ++it) {
      if (!complex_solve(n, M, v)) return false;
      R nv = 0;
      for (const C &x : v) nv += std::norm(x);
      nv = std::sqrt(nv);
      // fix the phase so that a real eigenvector comes out real
      int big = 0;
      for (int i = 1; i < n; ++i)
        if (std::abs(v[i]) > std::abs(v[big])) big = i;
      const C ph = std::abs(v[big]) / v[big];
      for (C &x : v) x *= ph / nv;
    }
    if (!pair[u])
      for (C &x : v) x = C(x.real(), 0);
    vcol[u] = col;
    for (int i = 0; i < n; ++i) V[(size_t)i * n + col] = v[i];
    ++col;
    if (pair[u]) {
      for (int i = 0; i < n; ++i) V[(size_t)i * n + col] = std::conj(v[i]);
      ++col;
    }
  }
  // P = (B V)^{-1}: solve (B V) P = I column by column
  std::vector<C> BV((size_t)n * n, C(0));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      C s(0);
      for (int k = 0; k < n; ++k) s += B[(size_t)i * n + k] * V[(size_t)k * n + j];
      BV[(size_t)i * n + j] = s;
    }
  std::vector<C> P((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    std::vector<C> e(n, C(0));
    e[j] = C(1);
    if (!complex_solve(n, BV, e)) return false;
    for (int i = 0; i < n; ++i) P[(size_t)i * n + j] = e[i];
  }
  const int nu = (int)uniq.size();
  out.nq = n;
  out.nu = nu;
  out.lam.assign(2 * (size_t)nu, 0.0);
  out.fin.assign(2 * (size_t)nu * n, 0.0);
  out.fout.assign(2 * (size_t)n * nu, 0.0);
  out.ain.assign(2 * (size_t)nu * n, 0.0);
  out.aout.assign(2 * (size_t)n * nu, 0.0);
  for (int u = 0; u < nu; ++u) {
    out.lam[2 * u] = (double)uniq[u].real();
    out.lam[2 * u + 1] = (double)uniq[u].imag();
    const int c = vcol[u];
    const R w = pair[u] ? 2 : 1;  // a pair contributes 2 Re(.)
    for (int j = 0; j < n; ++j) {
      const C fi = P[(size_t)c * n + j], fo = w * V[(size_t)j * n + c];
      const C ai = V[(size_t)j * n + c], ao = w * P[(size_t)c * n + j];
      out.fin[2 * ((size_t)u * n + j)] = (double)fi.real();
      out.fin[2 * ((size_t)u * n + j) + 1] = (double)fi.imag();
      out.fout[2 * ((size_t)j * nu + u)] = (double)fo.real();
      out.fout[2 * ((size_t)j * nu + u) + 1] = (double)fo.imag();
      out.ain[2 * ((size_t)u * n + j)] = (double)ai.real();
      out.ain[2 * ((size_t)u * n + j) + 1] = (double)ai.imag();
      out.aout[2 * ((size_t)j * nu + u)] = (double)ao.real();
      out.aout[2 * ((size_t)j * nu + u) + 1] = (double)ao.imag();
    }
  }
  return true;
}

}  // namespace sg
