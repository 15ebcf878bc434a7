// Double-double arithmetic for the host-side tables (about 32 significant
// digits).  Error-free transformations with std::fma; Dekker/Knuth style.
// Contraction is switched off inside every helper: fusing a rounded product
// into a later addition breaks the error-free transformations.
#pragma once

#include <cmath>

namespace sg {

struct ddv {
  double hi = 0.0, lo = 0.0;
  ddv() = default;
  ddv(double h) : hi(h), lo(0.0) {}
  ddv(double h, double l) : hi(h), lo(l) {}
  double value() const { return hi + lo; }
};

inline ddv quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return {s, b - (s - a)};
}
inline ddv two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
inline ddv two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return {p, std::fma(a, b, -p)};
}
inline ddv operator+(ddv a, ddv b) {
#pragma clang fp contract(off)
  ddv s = two_sum(a.hi, b.hi);
  ddv t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
inline ddv operator-(ddv a) { return {-a.hi, -a.lo}; }
inline ddv operator-(ddv a, ddv b) { return a + (-b); }
inline ddv operator*(ddv a, ddv b) {
#pragma clang fp contract(off)
  ddv p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}
inline ddv operator/(ddv a, ddv b) {
#pragma clang fp contract(off)
  const double q1 = a.hi / b.hi;
  ddv r = a - b * ddv(q1);
  const double q2 = r.hi / b.hi;
  r = r - b * ddv(q2);
  const double q3 = r.hi / b.hi;
  return ddv(q1) + ddv(q2) + ddv(q3);
}
inline ddv &operator+=(ddv &a, ddv b) { return a = a + b; }

// e^{-x} for 0 <= x <= 1 by its Taylor series (terms below 1e-34 dropped)
inline ddv exp_neg(ddv x) {
  ddv sum(1.0), term(1.0);
  for (int k = 1; k < 60; ++k) {
    term = term * x / ddv((double)k);
    term = -term;
    sum += term;
    if (std::fabs(term.hi) < 1e-34) break;
  }
  return sum;
}

// a^n by binary powering
inline ddv dd_pow(ddv a, long long n) {
  ddv r(1.0);
  while (n > 0) {
    if (n & 1) r = r * a;
    a = a * a;
    n >>= 1;
  }
  return r;
}

// I_k(lam) = int_0^1 s^k e^{-lam s} ds = sum_m (-lam)^m / (m! (k+m+1)),  0 <= lam <= 1
inline ddv moment(int k, ddv lam) {
  ddv sum(0.0), pw(1.0);  // pw = (-lam)^m / m!
  for (int m = 0; m < 80; ++m) {
    const ddv t = pw / ddv((double)(k + m + 1));
    sum += t;
    if (m > 2 && std::fabs(t.hi) < 1e-35) break;
    pw = -(pw * lam) / ddv((double)(m + 1));
  }
  return sum;
}

}  // namespace sg
