"""Spatial matrices (oracle; test infrastructure).

Eq. (9) pairs the time factors with two spatial bilinear forms on
V^x_{jx} subset of H^1_0(Omega):

    M[k,l] = (phi_l, phi_k)_{L^2(Omega)},
    K[k,l] = (c^2 grad phi_l, grad phi_k)_{L^2(Omega)}.

Omega = (0,len_0) in 1-D (P1 hats) or (0,len_0)x(0,len_1) in 2-D (Q1 hats,
x fastest in every flattened index).  The wave speed c is piecewise constant
on a uniform block grid of ncell cells per axis (blocks need not align with
coarse meshes).  On a block R = X_b x Y_b the integrand of K separates, so

    K = sum_blocks c_b^2 [ M^y(Y_b) (x) K^x(X_b) + K^y(Y_b) (x) M^x(X_b) ]

where M^x(X_b), K^x(X_b) are the 1-D mass/stiffness integrals restricted to
the interval X_b.  Every 1-D integral is evaluated exactly, in rational
arithmetic on the binary values of the lengths and speeds: the element is
split at the block edges and each piece [s_a, s_b] (element coordinate
s = x - x_e in [0, h], hats 1 - s/h and s/h) contributes the closed-form
integrals of the hat products and of their constant slopes +-1/h.  In 1-D
the sum over blocks is also exact and every entry is rounded once; in 2-D
the exact 1-D factors are rounded and combined in floating point.

Rounding once matters: K of a level has zero row sums inside a block, and a
few-ulp error per entry (as a floating-point quadrature gives) acts like a
reaction term of relative size ~eps/h^2, which the solution of the long time
levels shows at the 1e-13 level.
"""

import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

from . import basis



class Medium:
    """Piecewise-constant wave speed on a uniform block grid.

    lengths: domain side lengths (d entries); ncell: blocks per axis;
    c_vals: block values, x fastest.
    """

    def __init__(self, lengths, ncell, c_vals):
        self.d = len(lengths)
        self.lengths = [float(v) for v in lengths]
        self.ncell = [int(v) for v in ncell]
        self.c = np.asarray(c_vals, dtype=np.float64).reshape(
            list(reversed(self.ncell)))  # [ny][nx] in 2-D
        if np.any(self.c <= 0) or not np.all(np.isfinite(self.c)):
            raise ValueError("wave speed must be positive and finite")

    def block_interval(self, axis, b):
        """Block b's interval along `axis` as exact Fractions."""
        w = Fraction(self.lengths[axis]) / self.ncell[axis]
        return b * w, (b + 1) * w


def _pieces_1d(j, length, lo, hi):
    """Exact 1-D P1 mass and unit-stiffness integrals over [lo, hi] (Fractions):
    dict (row, col) -> [m, k] over interior indices, n = 2^j elements."""
    n = 2 ** j
    h = Fraction(length) / n
    out = {}
    e0 = max(0, math.floor(lo / h))
    e1 = min(n, math.ceil(hi / h))
    for e in range(e0, e1):
        xe = e * h
        a, b = max(lo, xe), min(hi, xe + h)
        if b <= a:
            continue
        ua, ub = (a - xe) / h, (b - xe) / h      # piece in units of h
        d1, d2, d3 = ub - ua, ub ** 2 - ua ** 2, ub ** 3 - ua ** 3
        # int (1-u)^2, int u (1-u), int u^2 over [ua, ub], times h; slopes -+1/h
        mass_loc = {(e, e): h * (d1 - d2 + d3 / 3), (e, e + 1): h * (d2 / 2 - d3 / 3),
                    (e + 1, e + 1): h * d3 / 3}
        k_abs = d1 / h
        for p in (e, e + 1):
            for q in (e, e + 1):
                if not (1 <= p <= n - 1 and 1 <= q <= n - 1):
                    continue
                m = mass_loc[(min(p, q), max(p, q))]
                k = k_abs if p == q else -k_abs
                acc = out.setdefault((p - 1, q - 1), [Fraction(0), Fraction(0)])
                acc[0] += m
                acc[1] += k
    return out


def _to_csr(entries, which, n, scale=None):
    rows = [r for r, _ in entries]
    cols = [c for _, c in entries]
    vals = [float(v[which] if scale is None else v[which] * scale) for v in entries.values()]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n - 1, n - 1))


def _matrices_1d_on(j, length, lo, hi):
    """1-D P1 mass and unit stiffness integrated over [lo,hi] only, each entry
    the rounded exact integral.  Returns (M, K), sparse (n-1)x(n-1), n = 2^j."""
    e = _pieces_1d(j, length, Fraction(lo), Fraction(hi))
    return _to_csr(e, 0, 2 ** j), _to_csr(e, 1, 2 ** j)


def mass_1d(j, length):
    return _matrices_1d_on(j, length, 0.0, length)[0]


def mass(j, medium):
    """Mass matrix of V^x_j (P1 in 1-D, Q1 = Kronecker product in 2-D)."""
    if medium.d == 1:
        return mass_1d(j, medium.lengths[0])
    return sp.kron(mass_1d(j, medium.lengths[1]), mass_1d(j, medium.lengths[0]),
                   format="csr")


def _stiff_exact_1d(j, medium):
    """1-D stiffness entries as exact Fractions: dict (row, col) -> value."""
    acc = {}
    for bx in range(medium.ncell[0]):
        lo, hi = medium.block_interval(0, bx)
        c2 = Fraction(float(medium.c[bx])) ** 2
        for key, (_, k) in _pieces_1d(j, medium.lengths[0], lo, hi).items():
            acc[key] = acc.get(key, Fraction(0)) + c2 * k
    return acc


def _split_csr(entries, shape):
    """(hi, lo) CSR matrices of exact entries, hi = rounded value, lo = the
    rounded remainder; both with the same sparsity pattern."""
    keys = sorted(entries)
    rows = [r for r, _ in keys]
    cols = [c for _, c in keys]
    hi = [float(entries[k]) for k in keys]
    lo = [float(entries[k] - Fraction(h)) for k, h in zip(keys, hi)]
    mk = lambda v: sp.csr_matrix((v, (rows, cols)), shape=shape)
    return mk(hi), mk(lo)


def stiff_lo(j, medium):
    """K - stiff(j, medium) rounded (1-D; the exact entries are hi + lo to
    ~32 digits).  None in 2-D, where the entries are formed in floating point."""
    if medium.d != 1:
        return None
    n = 2 ** j
    return _split_csr(_stiff_exact_1d(j, medium), (n - 1, n - 1))[1]


def stiff(j, medium):
    """Stiffness matrix (c^2 grad u, grad v) of V^x_j, exact in c^2."""
    if medium.d == 1:
        # sum over blocks in exact arithmetic, one rounding per entry
        n = 2 ** j
        return _split_csr(_stiff_exact_1d(j, medium), (n - 1, n - 1))[0]
    Lx, Ly = medium.lengths
    xs = [_matrices_1d_on(j, Lx, *medium.block_interval(0, b))
          for b in range(medium.ncell[0])]
    ys = [_matrices_1d_on(j, Ly, *medium.block_interval(1, b))
          for b in range(medium.ncell[1])]
    K = None
    for by in range(medium.ncell[1]):
        My, Ky = ys[by]
        for bx in range(medium.ncell[0]):
            Mx, Kx = xs[bx]
            part = medium.c[by, bx] ** 2 * (sp.kron(My, Kx) + sp.kron(Ky, Mx))
            K = part if K is None else K + part
    return K.tocsr()


def cross_stiff_1d(a, J, medium):
    """(Phi^T K^J)[k, m] = (c^2 phi^J_m', phi^a_k') in 1-D, each entry the
    rounded exact value.  On fine element e both slopes are constant, so
    the entry is (C_{m-1} s_k(m-1) - C_m s_k(m)) / h_J with C_e the exact
    integral of c^2 over element e and s_k(e) the slope of the coarse hat k
    there (+-1/h_a or 0): nonzero only at coarse nodes and at block edges."""
    n, na = 2 ** J, 2 ** a
    ratio = n // na
    L0 = Fraction(medium.lengths[0])
    hJ, ha = L0 / n, L0 / na
    C = [Fraction(0)] * n
    for bx in range(medium.ncell[0]):
        lo, hi = medium.block_interval(0, bx)
        c2 = Fraction(float(medium.c[bx])) ** 2
        for e in range(max(0, math.floor(lo / hJ)), min(n, math.ceil(hi / hJ))):
            ov = min(hi, (e + 1) * hJ) - max(lo, e * hJ)
            if ov > 0:
                C[e] += c2 * ov

    def slope(k, e):
        E = e // ratio           # coarse element holding fine element e
        return 1 / ha if E == k - 1 else (-1 / ha if E == k else 0)

    rows, cols, vals = [], [], []
    for k in range(1, na):
        for m in range((k - 1) * ratio, (k + 1) * ratio + 1):
            if not 1 <= m <= n - 1:
                continue
            v = (C[m - 1] * slope(k, m - 1) - C[m] * slope(k, m)) / hJ
            if v != 0:
                rows.append(k - 1)
                cols.append(m - 1)
                vals.append(float(v))
    return sp.csr_matrix((vals, (rows, cols)), shape=(na - 1, n - 1))


def interp_1d(a, J, length):
    """Phi[m, k] = phi^a_k(x^J_m): nodal values of level-a hats on level J."""
    xs = (length / 2 ** J) * np.arange(1, 2 ** J)
    ratio = 2 ** (J - a)
    rows, cols, vals = [], [], []
    for k in range(1, 2 ** a):
        # fine nodes inside the support (x_{k-1}, x_{k+1}) of the coarse hat
        m = np.arange((k - 1) * ratio + 1, (k + 1) * ratio)
        v = basis.hat_1d_node(a, length, k, xs[m - 1])
        rows.extend(m - 1)
        cols.extend([k - 1] * len(m))
        vals.extend(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 ** J - 1, 2 ** a - 1))


def interp(a, J, medium):
    """Prolongation V^x_a -> V^x_J as a matrix on nodal values (exact, nested)."""
    if medium.d == 1:
        return interp_1d(a, J, medium.lengths[0])
    return sp.kron(interp_1d(a, J, medium.lengths[1]),
                   interp_1d(a, J, medium.lengths[0]), format="csr")
