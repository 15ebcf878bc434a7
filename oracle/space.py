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
the interval X_b.  Every 1-D integral is evaluated element by element after
splitting the element at the block edges, with a 3-point Gauss-Legendre rule
(exact for the piecewise-quadratic integrands).

Cross-level matrices use nesting (Sec. 2.2: V_{jx} subset of V_{jx+1}):
a coarse hat is the combination of fine hats with its nodal values,
phi^a_k = sum_m phi^a_k(x_m) phi^J_m, so (phi^J_m, phi^a_k) = (Phi^T M^J)[k,m].
"""

import numpy as np
import scipy.sparse as sp

from . import basis

_GX, _GW = np.polynomial.legendre.leggauss(3)


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
        w = self.lengths[axis] / self.ncell[axis]
        return b * w, (b + 1) * w


def _matrices_1d_on(j, length, lo, hi):
    """1-D P1 mass and unit stiffness integrated over [lo,hi] only.

    Returns (M, K) as sparse (n-1)x(n-1) matrices, n = 2^j."""
    n = 2 ** j
    h = length / n
    rows, cols, mv, kv = [], [], [], []
    e0 = max(0, int(np.floor(lo / h)) - 1)
    e1 = min(n, int(np.ceil(hi / h)) + 1)
    for e in range(e0, e1):
        a, b = max(lo, e * h), min(hi, (e + 1) * h)
        if b <= a:
            continue
        xs = 0.5 * (b - a) * _GX + 0.5 * (a + b)
        ws = 0.5 * (b - a) * _GW
        # the element's two nodes are e and e+1 (interior index = node - 1)
        nodes = [k for k in (e, e + 1) if 1 <= k <= n - 1]
        phi = {k: basis.hat_1d_node(j, length, k, xs) for k in nodes}
        dphi = {k: basis.hat_1d_node_deriv(j, length, k, xs) for k in nodes}
        for p in nodes:
            for q in nodes:
                rows.append(p - 1)
                cols.append(q - 1)
                mv.append(np.sum(ws * phi[p] * phi[q]))
                kv.append(np.sum(ws * dphi[p] * dphi[q]))
    shape = (n - 1, n - 1)
    return (sp.csr_matrix((mv, (rows, cols)), shape=shape),
            sp.csr_matrix((kv, (rows, cols)), shape=shape))


def mass_1d(j, length):
    return _matrices_1d_on(j, length, 0.0, length)[0]


def mass(j, medium):
    """Mass matrix of V^x_j (P1 in 1-D, Q1 = Kronecker product in 2-D)."""
    if medium.d == 1:
        return mass_1d(j, medium.lengths[0])
    return sp.kron(mass_1d(j, medium.lengths[1]), mass_1d(j, medium.lengths[0]),
                   format="csr")


def stiff(j, medium):
    """Stiffness matrix (c^2 grad u, grad v) of V^x_j, exact in c^2."""
    if medium.d == 1:
        L0 = medium.lengths[0]
        K = None
        for bx in range(medium.ncell[0]):
            lo, hi = medium.block_interval(0, bx)
            part = medium.c[bx] ** 2 * _matrices_1d_on(j, L0, lo, hi)[1]
            K = part if K is None else K + part
        return K.tocsr()
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
