// Host-side tables of the discrete operator (time matrices, tap tables,
// spatial eigenvalues, sine transforms).  Pure C++, no HIP calls.
#pragma once

#include <vector>

namespace sg {

// Gauss-Legendre nodes/weights on [-1,1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

// Quadratic C^1 B-splines on the clamped uniform knot vector of level b of
// (0,T), basis psi_i = B_{i+1}, i = 0..2^b.  On element e (t in
// [e h, (e+1) h]) the nonzero functions are B_e, B_{e+1}, B_{e+2}; these
// return their values / first / second derivatives at t in v[0..2].
void spline_local(int b, double T, int e, double t, double v[3], double d1[3],
                  double d2[3]);

struct TimeLevel {
  int b = 0, nq = 0;
  std::vector<double> A, B;      // banded [nq][5], column j-i+2 (high parts)
  std::vector<double> Alo, Blo;  // low parts: A = A + Alo exactly to ~32 digits
  std::vector<double> Dlo, Dhi;  // psi_i'(t_i), psi_i'(t_{i+1})
  std::vector<double> g;         // int psi_i' e^{-t/T}
  double d0 = 0;                 // psi_0'(0) (psi_i'(0) = 0 for i > 0)
};

// Time matrices of Prop. 1 / eq. (30) for level b:
//   A[i][j] = (psi_j'', psi_i')_{L2_e} + psi_j'(0) psi_i'(0),
//   B[i][j] = (psi_j, psi_i')_{L2_e},   weight e^{-t/T},
// from exact moment integrals in double-double (see tables.cpp).
TimeLevel time_level(int b, double T);

// Tap tables on the finest time grid (level J): for each fine node n,
// q0[n] and w[3n..3n+2] such that the coupling of slab n to time index q is
// w[k] for q = q0[n]+k.
struct Taps {
  std::vector<int> q0;
  std::vector<double> w;
};
// P1 taps of level b: (Lambda_b^T M_e)[q][n], M_e the weighted P1 mass on
// the fine time grid, Lambda_b the P1 hats of level b at fine nodes.
Taps p1_taps(int b, int J, double T);
// Spline taps of level b: psi^b_q(t_n).
Taps spline_taps(int b, int J, double T);
// Spline taps of level b at arbitrary instants t[n] in [0,T]: psi^b_q(t_n)
// (deriv = 0) or psi^b_q'(t_n) (deriv = 1).
Taps spline_taps_at(int b, double T, const std::vector<double> &t, int deriv);
// Time-sum taps: q0 = 0, w = (1,0,0) for every n (sum over slabs).
Taps sum_taps(int J);

// 1-D P1 eigenvalues on (0,len) at level a (unit wave speed):
// m_k = h/6 (4 + 2 cos(k pi/n)), kappa_k = 4/h sin^2(k pi/(2n)), k = 1..n-1.
void p1_eigen(int a, double len, std::vector<double> &m, std::vector<double> &k);

// Variable wave speed (d = 1): average of c^2 over every element of level a
// of (0, len) for c piecewise constant on ncell uniform blocks.
std::vector<double> element_c2(int a, double len, int ncell, const double *c_vals);
// Generalised eigenpairs of the level-a P1 pencil (K(c), M): K V = M V diag(lam),
// V^T M V = I.  V is row-major (n-1)^2, column k = eigenvector k.  c2e holds the
// element averages of c^2 (2^a values).
void pencil_eigen(int a, double len, const std::vector<double> &c2e, std::vector<double> &V,
                  std::vector<double> &lam);

// Dense Q1 pencil of level a in 2-D (n = 2^a - 1 nodes per axis, x fastest):
// K(c) and M, both row-major n^2 x n^2 and symmetric, on (0,len[0]) x
// (0,len[1]) with c piecewise constant on ncell[0] x ncell[1] uniform blocks
// (x fastest).  Every element integral is taken exactly over the part of the
// element inside each block (in long double) and rounded once.
void pencil_2d(int a, const double *len, const int *ncell, const double *c_vals,
               std::vector<double> &K, std::vector<double> &M);

// c^2-weighted 1-D P1 stiffness and mass of level a on (0, len) for c
// piecewise constant on ncell uniform blocks (c_row: the block values), each
// entry integrated exactly over the parts of its elements in every block:
// [4][n] = K diagonal, K coupling (k, k+1), M diagonal, M coupling (k, k+1),
// n = 2^a - 1 (coupling entries 0 at the last node).  One strip of 2-D
// wave-speed blocks, whose speed depends on x only.
std::vector<double> strip_x_tables(int a, double len, int ncell, const double *c_row);

// Tridiagonal M and K(c) of level a (d = 1) per interior node k, kSpaceStride
// doubles: [M_kk, M_{k,k+1}, K_kk, K_{k,k+1}, lo(K_kk), lo(K_{k,k+1})] (the
// coupling entries are 0 at the last node).  K is formed in double-double
// from the block speeds and split as hi + lo: inside a block its rows sum to
// zero, and the rounding of a diagonal entry alone would act as a reaction
// term of relative size ~eps/h^2 on the smooth modes.
constexpr int kSpaceStride = 6;
std::vector<double> space_entries(int a, double len, int ncell, const double *c_vals);
// Block LU of the component matrix S = A (x) M + B (x) K in space-major
// order (block k = the time values at spatial node k): D_0 = S_00,
// L_k = S_{k,k-1} D_{k-1}^{-1}, D_k = S_kk - L_k S_{k-1,k}.  Computed in
// extended precision from the double-double time matrices; outputs Dinv[k]
// = D_k^{-1} and Lf[k] = L_k (row-major nq x nq each, Lf[0] unused).
void block_lu(const TimeLevel &tl, const std::vector<double> &mk, int nx,
              std::vector<double> &Dinv, std::vector<double> &Lf);

// Diagonalisation of a short time level (fast diagonalisation in time):
// B^{-1} A = V diag(lam) V^{-1}, A and B the time matrices of Prop. 1, in
// extended precision (Hessenberg reduction, shifted complex QR, inverse
// iteration).  The spectrum of a real pencil is closed under conjugation;
// only the real eigenvalues and one member (Im > 0) of each conjugate pair
// are kept, nu in all.  With P = (B V)^{-1} the component system
// S = A (x) M + B (x) K is solved as
//   forward:  r_u = sum_j fin[u][j] b_j,   (lam_u M + K) w_u = r_u,
//             u_j = Re sum_u fout[j][u] w_u;
//   adjoint (S^T z = y): r_u = sum_j ain[u][j] y_j, the same spatial
//             systems, z_j = Re sum_u aout[j][u] w_u;
// fin/ain are P's and V^T's rows, fout/aout V's and P^T's columns, times 2
// for a conjugate pair (its partner contributes the conjugate).  Complex
// values are interleaved (re, im).  Returns false if the iteration fails.
struct TimeFdm {
  int nq = 0, nu = 0;
  std::vector<double> lam;         // [nu] complex
  std::vector<double> fin, ain;    // [nu][nq] complex
  std::vector<double> fout, aout;  // [nq][nu] complex
};
bool time_fdm(const TimeLevel &tl, TimeFdm &out);

// Orthonormal DST-I matrix of level a: Q[j][k] = sqrt(2/n) sin(pi j k/n),
// j,k = 1..n-1, n = 2^a (symmetric, Q Q = I), row-major (n-1)^2.
std::vector<double> dst_matrix(int a);

}  // namespace sg
