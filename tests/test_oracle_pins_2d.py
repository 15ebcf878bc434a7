"""Pins of the oracle's 2-D data path and of its full-grid solve.

Every expected value here comes from an independent evaluation of the
paper's definitions: the right-hand side of eq. (9) for the interpolated
nodal data by a tensor Gauss quadrature on a space-time sub-grid that
refines the finest mesh and the wave-speed blocks; nodal prolongation by
closed-form hat values; the Q1 mass matrix by quadrature; the full-grid
Galerkin solution P_{j,j} (eq. 10 on V_j (x) V_j) from a dense system whose
entries are the bilinear form (6) evaluated by quadrature.  The domain is
not square (1.0 x 0.8) and the 3 x 2 speed blocks are not aligned with the
meshes, so a swap of the axes or of a Kronecker order changes the result.
"""

import numpy as np
import pytest

from oracle import Problem, basis

LX, LY = 1.0, 0.8
NCX, NCY = 3, 2


def _pieces(length, nmesh, ncell, npts=3):
    """Gauss points and weights on the sub-intervals of (0, length) cut at the
    level-nmesh mesh nodes and at the block edges."""
    br = np.unique(np.concatenate([length * np.arange(nmesh + 1) / nmesh,
                                   length * np.arange(ncell + 1) / ncell]))
    g, gw = np.polynomial.legendre.leggauss(npts)
    a, b = br[:-1], br[1:]
    pts = (0.5 * (a + b)[:, None] + 0.5 * (b - a)[:, None] * g[None, :]).reshape(-1)
    wts = (0.5 * (b - a)[:, None] * gw[None, :]).reshape(-1)
    return pts, wts


def _time_points(J, T, npts=8):
    nf = 2 ** J
    g, gw = np.polynomial.legendre.leggauss(npts)
    tq = ((np.arange(nf)[:, None] + 0.5 + 0.5 * g) * T / nf).reshape(-1)
    tw = np.tile(0.5 * gw, nf) * T / nf
    return tq, tw


def _hat(s):
    return np.maximum(0.0, 1.0 - np.abs(s))


def _hats(j, length, x):
    """(len(x), 2^j - 1) values of the level-j interior hats, closed form."""
    h = length / 2 ** j
    k = np.arange(1, 2 ** j)
    return _hat((np.asarray(x)[:, None] - k[None, :] * h) / h)


def _hats_deriv(j, length, x):
    h = length / 2 ** j
    k = np.arange(1, 2 ** j)
    s = (np.asarray(x)[:, None] - k[None, :] * h) / h
    return np.where(np.abs(s) < 1.0, -np.sign(s) / h, 0.0)


class _Quad2D:
    """Quadrature grid on (0,LX) x (0,LY) for meshes up to level J."""

    def __init__(self, J, cv):
        self.xq, self.xw = _pieces(LX, 2 ** J, NCX)
        self.yq, self.yw = _pieces(LY, 2 ** J, NCY)
        bx = np.minimum((self.xq / (LX / NCX)).astype(int), NCX - 1)
        by = np.minimum((self.yq / (LY / NCY)).astype(int), NCY - 1)
        self.c2 = np.asarray(cv).reshape(NCY, NCX)[by[:, None], bx[None, :]] ** 2
        self.W = self.yw[:, None] * self.xw[None, :]

    def basis(self, j):
        return (_hats(j, LX, self.xq), _hats_deriv(j, LX, self.xq),
                _hats(j, LY, self.yq), _hats_deriv(j, LY, self.yq))

    def field(self, J, u):
        """Values, x- and y-derivatives of the level-J Q1 interpolant of u."""
        px, dpx, py, dpy = self.basis(J)
        U = np.asarray(u).reshape(2 ** J - 1, 2 ** J - 1)
        return py @ U @ px.T, py @ U @ dpx.T, dpy @ U @ px.T

    def project(self, j, V, Vx=None, Vy=None):
        """int V phi_k, or (V None) int c^2 (Vx d_x phi_k + Vy d_y phi_k), over
        Omega for the level-j hats, flattened x fastest."""
        px, dpx, py, dpy = self.basis(j)
        if Vx is None:
            out = py.T @ (self.W * V) @ px
        else:
            out = (py.T @ (self.W * self.c2 * Vx) @ dpx + dpy.T @ (self.W * self.c2 * Vy) @ px)
        return out.reshape(-1)

    def mass(self, j):
        px, _, py, _ = self.basis(j)
        Mx = px.T @ (self.xw[:, None] * px)
        My = py.T @ (self.yw[:, None] * py)
        n = px.shape[1]
        M = np.zeros((n * n, n * n))
        for ky in range(n):
            for kx in range(n):
                for ly in range(n):
                    for lx in range(n):
                        M[ky * n + kx, ly * n + lx] = My[ky, ly] * Mx[kx, lx]
        return M

    def stiff(self, j):
        px, dpx, py, dpy = self.basis(j)
        n = px.shape[1]
        K = np.zeros((n * n, n * n))
        for ky in range(n):
            for kx in range(n):
                a = self.c2 * (np.outer(py[:, ky], dpx[:, kx]) * self.W)
                b = self.c2 * (np.outer(dpy[:, ky], px[:, kx]) * self.W)
                K[ky * n + kx] = (py.T @ a @ dpx + dpy.T @ b @ px).reshape(-1)
        return K


def _brute_load_2d(prob, q, jx, jt, f, u0, v0):
    """Right-hand side of eq. (9) on V_jx (x) V_jt for the P1-in-time /
    Q1-in-space interpolants of the nodal data (quadrature)."""
    J, T = prob.J, prob.T
    tq, tw = _time_points(J, T)
    lam = basis.p1_time_hat(J, T, tq)                    # (tq, 2^J + 1)
    px, _, py, _ = q.basis(J)
    F = np.einsum("tn,nyx->tyx", lam, f)
    F = np.einsum("tyx,Yy,Xx->tYX", F, py, px)           # interpolant at (t, y, x)
    dps = basis.time_basis(jt, T, tq, 1) * (tw * np.exp(-tq / T))[:, None]
    d0 = basis.time_basis(jt, T, np.array([0.0]), 1)[0]
    cx, _, cy, _ = q.basis(jx)
    P = np.einsum("tYX,YX,Xk,Yl->tlk", F, q.W, cx, cy).reshape(len(tq), -1)
    b = dps.T @ P
    V, _, _ = q.field(J, v0)
    b += np.outer(d0, q.project(jx, V))
    _, Ux, Uy = q.field(J, u0)
    b -= np.outer(dps.sum(axis=0), q.project(jx, None, Ux, Uy))
    return b


def _problem_2d(L, seed):
    rng = np.random.default_rng(seed)
    cv = rng.uniform(0.5, 2.0, NCX * NCY)
    prob = Problem(2, [LX, LY], [NCX, NCY], cv, 1.0, L)
    n = 2 ** prob.J - 1
    f = rng.standard_normal((prob.nt_fine, n, n))
    u0 = rng.standard_normal((n, n))
    v0 = rng.standard_normal((n, n))
    return prob, cv, f, u0, v0


def test_load_matches_rhs_eq9_2d():
    """b_c of every component equals the right-hand side of eq. (9) for the
    interpolated nodal data on a non-square domain with 3 x 2 speed blocks
    that the meshes do not resolve (quadrature on a sub-grid cut at the
    mesh nodes and block edges)."""
    prob, cv, f, u0, v0 = _problem_2d(4, 21)
    q = _Quad2D(prob.J, cv)
    for jx, jt, _ in prob.comps:
        b = _brute_load_2d(prob, q, jx, jt, f, u0, v0)
        bo = prob.load(jx, jt, f, u0, v0)
        assert bo.shape == b.shape
        assert np.abs(bo - b).max() <= 1e-12 * np.abs(b).max(), (jx, jt)


def test_load_2d_each_datum_separately():
    """The three terms of eq. (9) one at a time (f only, v0 only, u0 only):
    a sign or a term attached to the wrong datum fails here even where the
    sum might mask it."""
    prob, cv, f, u0, v0 = _problem_2d(4, 22)
    q = _Quad2D(prob.J, cv)
    z, zt = np.zeros_like(u0), np.zeros_like(f)
    for data in ((f, z, z), (zt, u0, z), (zt, z, v0)):
        for jx, jt in ((2, 2), (3, 1), (1, 3)):
            b = _brute_load_2d(prob, q, jx, jt, *data)
            bo = prob.load(jx, jt, *data)
            assert np.abs(bo - b).max() <= 1e-12 * np.abs(b).max(), (jx, jt)


def test_interp_2d_hat_values():
    """Phi[(m_y, m_x), (k_y, k_x)] = phi_kx(x_mx) phi_ky(y_my) on a
    non-square domain, from closed-form hat values (x fastest)."""
    prob, *_ = _problem_2d(5, 23)
    J = prob.J
    xs = LX * np.arange(1, 2 ** J) / 2 ** J
    ys = LY * np.arange(1, 2 ** J) / 2 ** J
    for a in (1, 2, 4):
        P = prob.phi(a).toarray()
        hx = _hats(a, LX, xs)
        hy = _hats(a, LY, ys)
        n, na = 2 ** J - 1, 2 ** a - 1
        ref = np.einsum("yl,xk->yxlk", hy, hx).reshape(n * n, na * na)
        assert np.abs(P - ref).max() <= 4e-15


def test_mass_and_stiffness_2d_nonsquare():
    """Q1 mass (phi_l, phi_k) and stiffness (c^2 grad phi_l, grad phi_k) on
    (0,1) x (0,0.8) with non-aligned 3 x 2 blocks, entry by entry against
    quadrature.  Swapping the axes of the stiffness terms (M_x (x) K_y in
    place of M_y (x) K_x) fails since h_x != h_y; the mass is unchanged by
    that swap on a uniform mesh (both factors are multiples of one matrix)."""
    prob, cv, *_ = _problem_2d(4, 24)
    q = _Quad2D(prob.J, cv)
    for j in (1, 2, 3):
        M = prob.mass(j).toarray()
        K = prob.stiff(j).toarray()
        Mb, Kb = q.mass(j), q.stiff(j)
        assert np.abs(M - Mb).max() <= 1e-14 * np.abs(Mb).max(), j
        assert np.abs(K - Kb).max() <= 1e-12 * np.abs(Kb).max(), j


def _brute_time_forms(jt, T, J):
    """(psi_j'', psi_i')_e + psi_j'(0) psi_i'(0) and (psi_j, psi_i')_e by
    quadrature (weight e^{-t/T}); rows i, columns j."""
    tq, tw = _time_points(max(J, jt) + 2, T)
    ew = tw * np.exp(-tq / T)
    p0, p1, p2 = (basis.time_basis(jt, T, tq, k) for k in range(3))
    d0 = basis.time_basis(jt, T, np.array([0.0]), 1)[0]
    A = p1.T @ (ew[:, None] * p2) + np.outer(d0, d0)
    B = p1.T @ (ew[:, None] * p0)
    return A, B


def _brute_full_grid(prob, j, bload, space_mass, space_stiff, phi_fine, u0):
    """u0 + sum_{i,k} u[i,k] psi_i(t_n) phi_k(x_m) for the dense Galerkin
    solution u of the bilinear form (6) on V_j (x) V_j."""
    A, B = _brute_time_forms(j, prob.T, prob.J)
    nT, nX = A.shape[0], space_mass.shape[0]
    S = np.zeros((nT * nX, nT * nX))
    for i in range(nT):
        for jj in range(nT):
            S[i * nX:(i + 1) * nX, jj * nX:(jj + 1) * nX] = (A[i, jj] * space_mass
                                                            + B[i, jj] * space_stiff)
    u = np.linalg.solve(S, bload.reshape(-1)).reshape(nT, nX)
    tn = prob.T * np.arange(prob.nt_fine) / 2 ** prob.J
    psi = basis.time_basis(j, prob.T, tn, 0)
    return u0.reshape(1, -1) + psi @ u @ phi_fine.T


@pytest.mark.parametrize("j", [1, 2, 3])
def test_full_grid_2d_matches_dense_galerkin(j):
    """P_{j,j} + u0 on the finest grid (eq. 10 on V_j (x) V_j, the lift of
    Sec. 2.1) against the dense Galerkin solve of quadrature-built forms and
    load, evaluated at the fine nodes with closed-form hats."""
    prob, cv, f, u0, v0 = _problem_2d(4, 25)
    q = _Quad2D(prob.J, cv)
    b = _brute_load_2d(prob, q, j, j, f, u0, v0)
    J = prob.J
    xs = LX * np.arange(1, 2 ** J) / 2 ** J
    ys = LY * np.arange(1, 2 ** J) / 2 ** J
    n, nj = 2 ** J - 1, 2 ** j - 1
    phi = np.einsum("yl,xk->yxlk", _hats(j, LY, ys), _hats(j, LX, xs)).reshape(n * n, nj * nj)
    ref = _brute_full_grid(prob, j, b, q.mass(j), q.stiff(j), phi, u0.reshape(-1))
    got = prob.full_grid(j, f, u0, v0)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_full_grid_1d_matches_dense_galerkin():
    """As the 2-D pin, in 1-D with 3 speed blocks not aligned with the mesh."""
    rng = np.random.default_rng(26)
    cv = rng.uniform(0.5, 2.0, 3)
    length, T = 1.3, 0.9
    prob = Problem(1, [length], [3], cv, T, 5)
    J = prob.J
    n = 2 ** J - 1
    f = rng.standard_normal((prob.nt_fine, n))
    u0 = rng.standard_normal(n)
    v0 = rng.standard_normal(n)
    xq, xw = _pieces(length, 2 ** J, 3)
    c2 = cv[np.minimum((xq / (length / 3)).astype(int), 2)] ** 2
    tq, tw = _time_points(J, T)
    lam = basis.p1_time_hat(J, T, tq)
    phJ, dphJ = _hats(J, length, xq), _hats_deriv(J, length, xq)
    F = lam @ f @ phJ.T
    xs = length * np.arange(1, 2 ** J) / 2 ** J
    for j in (2, 4):
        ph, dph = _hats(j, length, xq), _hats_deriv(j, length, xq)
        dps = basis.time_basis(j, T, tq, 1) * (tw * np.exp(-tq / T))[:, None]
        d0 = basis.time_basis(j, T, np.array([0.0]), 1)[0]
        b = dps.T @ F @ (ph * xw[:, None])
        b += np.outer(d0, (phJ @ v0 * xw) @ ph)
        b -= np.outer(dps.sum(axis=0), (c2 * (dphJ @ u0) * xw) @ dph)
        Mj = ph.T @ (xw[:, None] * ph)
        Kj = dph.T @ ((c2 * xw)[:, None] * dph)
        ref = _brute_full_grid(prob, j, b, Mj, Kj, _hats(j, length, xs), u0)
        got = prob.full_grid(j, f, u0, v0)
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), j


@pytest.mark.parametrize("d", [1, 2])
def test_single_component_combination_is_the_full_grid(d):
    """At L = 2 the combination (eq. 19) has the single term (1,1) with sign
    +1, so the forward map equals P_{1,1} + u0."""
    rng = np.random.default_rng(27)
    if d == 1:
        prob = Problem(1, [1.0], [1], [1.3], 1.0, 2)
    else:
        prob = Problem(2, [LX, LY], [1, 1], [0.7], 1.0, 2)
    shape = prob.fine_shape()
    f = rng.standard_normal(shape)
    u0 = rng.standard_normal(shape[1:])
    v0 = rng.standard_normal(shape[1:])
    U = prob.forward(f, u0, v0)
    P = prob.full_grid(1, f, u0, v0)
    assert np.abs(U - P).max() <= 1e-14 * np.abs(P).max()
    assert np.allclose(U[0], u0.reshape(-1), atol=0, rtol=0)
