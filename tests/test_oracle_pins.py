"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them compares the oracle with
itself: identities of the paper (eqs. 2-3), textbook closed forms, brute-force
evaluation of the bilinear form (6) and load (9) by an independent space-time
quadrature, convergence rates (eq. 14, eq. 18, Theorem 1), the projector
exactness of the combination formula (eq. 19) and the telescoping identities
(eqs. 20-21).
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Problem, basis, levels, space, timemat
from oracle import method


# ---------------------------------------------------------------- levels --

@pytest.mark.parametrize("L", [2, 3, 6, 10, 14])
def test_component_set_eq19(L):
    """Eq. (19): 2J+1 solves with J = L-2, +1 on jx+jt = L, -1 on L-1."""
    comps = levels.components(L)
    J = L - 2
    assert len(comps) == 2 * J + 1
    assert sum(s for _, _, s in comps) == 1
    plus = {(a, b) for a, b, s in comps if s > 0}
    minus = {(a, b) for a, b, s in comps if s < 0}
    # paper indices (level - 1): +1 on jx' + jt' = J, -1 on jx' + jt' = J-1
    assert plus == {(jx + 1, J - jx + 1) for jx in range(0, J + 1)}
    assert minus == {(jx, J - jx + 1) for jx in range(1, J + 1)}


def test_sparse_dof_count_formula_d2():
    """Sec. 3.2, d=2: our count equals the sum of component dimensions, and
    the closed form of the paper (for dim V_j ~ 4^j, dim V_t ~ 2^j) is its
    leading-order behaviour."""
    assert levels.n_sparse(10, 2) == 1716413
    assert levels.n_full(10, 2) == 511 * 511 * 513
    assert levels.n_sparse(6, 1) == 439


# ---------------------------------------------------------------- time ----

@pytest.mark.parametrize("jt,T", [(1, 1.0), (2, 1.0), (3, 2.0), (5, 0.7), (7, 1.0)])
def test_time_matrix_identities_eq2_eq3(jt, T):
    """Weighted integration by parts, eqs. (2)-(3), applied to basis pairs:
    B + B^T = M_e/T + e_T e_T^T / e  and  A + A^T = K_e/T + d_T d_T^T/e + d_0 d_0^T
    (psi(0) = 0 for every basis function)."""
    tm = timemat.time_matrices(jt, T)
    A, B = tm["A"], tm["B"]
    lhs_b = B + B.T
    rhs_b = tm["Me"] / T + np.outer(tm["eT"], tm["eT"]) / math.e
    assert np.abs(lhs_b - rhs_b).max() <= 1e-13 * np.abs(rhs_b).max()
    lhs_a = A + A.T
    rhs_a = (tm["Ke"] / T + np.outer(tm["dT"], tm["dT"]) / math.e
             + np.outer(tm["d0"], tm["d0"]))
    assert np.abs(lhs_a - rhs_a).max() <= 1e-13 * np.abs(rhs_a).max()
    # Prop. 1: both have positive definite symmetric parts
    assert np.linalg.eigvalsh(0.5 * lhs_a).min() > 0
    assert np.linalg.eigvalsh(0.5 * lhs_b).min() > 0
    # pentadiagonal (quadratic B-splines overlap only with two neighbours)
    i, j = np.nonzero(np.abs(A) + np.abs(B))
    assert np.abs(i - j).max() <= 2


@pytest.mark.parametrize("jt,T", [(1, 1.0), (3, 1.3), (8, 2.0)])
def test_exact_time_matrices(jt, T):
    """The 32-digit time matrices satisfy eqs. (2)-(3) to 1e-30 (checked in
    40-digit arithmetic), agree with the independent double-precision
    quadrature to rounding, and their low parts are below half an ulp."""
    d = timemat.time_matrices_dd(jt, T)
    assert d["identity_A"] < 1e-30 and d["identity_B"] < 1e-30
    tm = timemat.time_matrices(jt, T)
    for name in ("A", "B"):
        hi = timemat.band_to_dense(d[name + "_hi"])
        lo = timemat.band_to_dense(d[name + "_lo"])
        assert np.abs(hi - tm[name]).max() <= 2e-15 * np.abs(tm[name]).max()
        assert np.all(np.abs(lo) <= 0.5 * np.spacing(np.abs(hi)) + 1e-300)


def test_long_time_solve_matches_40_digit_elimination():
    """N_t = 1025 (one spatial mode): the refined oracle solve equals a
    40-digit banded Gaussian elimination of the same system A m + B k."""
    import mpmath
    prob = Problem(1, [1.0], [1], [1.0], 1.0, 11)
    jx, jt = 1, 10
    rng = np.random.default_rng(21)
    b = rng.standard_normal((2 ** jt + 1, 1))
    x = prob.solve(jx, jt, b)[:, 0]
    m = prob.mass(jx).toarray()[0, 0]
    k = prob.stiff(jx).toarray()[0, 0]
    d = prob.tmat_dd(jt)
    n = 2 ** jt + 1
    with mpmath.workdps(40):
        M = [[mpmath.mpf(d["A_hi"][i, c]) + mpmath.mpf(d["A_lo"][i, c])
              for c in range(5)] for i in range(n)]
        Bm = [[mpmath.mpf(d["B_hi"][i, c]) + mpmath.mpf(d["B_lo"][i, c])
               for c in range(5)] for i in range(n)]
        S = [[M[i][c] * mpmath.mpf(m) + Bm[i][c] * mpmath.mpf(k) for c in range(5)]
             for i in range(n)]
        r = [mpmath.mpf(v) for v in b[:, 0]]
        for i in range(n):           # banded elimination, no pivoting
            for kk in (1, 2):
                if i + kk >= n:
                    continue
                lmul = S[i + kk][2 - kk] / S[i][2]
                for c in range(3):
                    S[i + kk][2 - kk + c] -= lmul * S[i][2 + c]
                r[i + kk] -= lmul * r[i]
        xs = [mpmath.mpf(0)] * n
        for i in range(n - 1, -1, -1):
            acc = r[i]
            for kk in (1, 2):
                if i + kk < n:
                    acc -= S[i][2 + kk] * xs[i + kk]
            xs[i] = acc / S[i][2]
        xr = np.array([float(v) for v in xs])
    assert np.linalg.norm(x - xr) <= 1e-13 * np.linalg.norm(xr)


def test_time_basis_textbook():
    """Clamped quadratic B-splines: partition of unity, only B_0 is nonzero at
    t=0, C^1 at interior knots, and on interior elements the uniform pieces
    (1-s)^2/2, (1+2s-2s^2)/2, s^2/2."""
    jt, T = 3, 1.0
    N = 2 ** jt
    h = T / N
    t = np.linspace(0, T, 97)
    full = basis.time_basis_full(jt, T, t)
    assert np.abs(full.sum(axis=1) - 1).max() < 1e-14
    assert np.abs(basis.time_basis(jt, T, np.array([0.0]))).max() == 0.0
    # C^1: derivative from the left and from the right agree at each knot
    for k in range(1, N):
        eps = 1e-9
        dl = basis.time_basis(jt, T, np.array([k * h - eps]), 1)
        dr = basis.time_basis(jt, T, np.array([k * h + eps]), 1)
        assert np.abs(dl - dr).max() < 1e-5
    # interior element e = 3: nonzero psi_{e-1}, psi_e, psi_{e+1}
    e = 3
    s = np.array([0.1, 0.5, 0.8])
    vals = basis.time_basis(jt, T, (e + s) * h)
    assert np.allclose(vals[:, e - 1], (1 - s) ** 2 / 2, atol=1e-15)
    assert np.allclose(vals[:, e], (1 + 2 * s - 2 * s ** 2) / 2, atol=1e-15)
    assert np.allclose(vals[:, e + 1], s ** 2 / 2, atol=1e-15)
    # the local evaluator agrees with the full recursion
    loc = timemat._span_values(jt, T, e, s, 1)[1]
    assert np.allclose(loc, basis.time_basis(jt, T, (e + s) * h, 1)[:, e - 1:e + 2])


def test_time_load_weights_reproduce_linear_data():
    """W applied to nodal values of 1 and of t integrates them exactly
    against psi_i' e^{-t/T} (P1 interpolation is exact for linear data)."""
    jt, J, T = 3, 6, 1.5
    W = timemat.load_weights(jt, J, T)
    tn = T * np.arange(2 ** J + 1) / 2 ** J
    tq, tw = method.fine_quadrature(J, T)
    dpsi = basis.time_basis(jt, T, tq, 1)
    w = tw * np.exp(-tq / T)
    assert np.allclose(W @ np.ones_like(tn), dpsi.T @ w, rtol=1e-13, atol=1e-14)
    assert np.allclose(W @ tn, dpsi.T @ (w * tq), rtol=1e-13, atol=1e-14)
    assert np.allclose(W @ (tn ** 2), dpsi.T @ (w * tq ** 2), rtol=1e-3)  # not exact
    assert not np.allclose(W @ (tn ** 2), dpsi.T @ (w * tq ** 2), rtol=1e-10)


def test_time_nodes_evaluation():
    """Psi at the finest nodes equals the Cox-de Boor values there."""
    jt, J, T = 2, 5, 1.0
    Psi = timemat.eval_at_nodes(jt, J, T)
    tn = T * np.arange(2 ** J + 1) / 2 ** J
    assert np.allclose(Psi, basis.time_basis(jt, T, tn), atol=1e-15)
    assert np.all(Psi[0] == 0)  # w(0) = 0 in V_t


# ---------------------------------------------------------------- space ---

def test_p1_matrices_textbook():
    """1-D P1, c = 1: M = h/6 tridiag(1,4,1), K = 1/h tridiag(-1,2,-1)."""
    j, length = 4, 2.0
    n = 2 ** j - 1
    h = length / 2 ** j
    med = space.Medium([length], [1], [1.0])
    M = space.mass(j, med).toarray()
    K = space.stiff(j, med).toarray()
    Mref = h / 6 * (4 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1))
    Kref = 1 / h * (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))
    assert np.abs(M - Mref).max() < 1e-15
    assert np.abs(K - Kref).max() < 1e-12


def test_q1_stencils_textbook():
    """2-D Q1 on a uniform square mesh, c = 1: the interior stencils are
    h^2/36 [1 4 1; 4 16 4; 1 4 1] (mass) and 1/3 [-1 -1 -1; -1 8 -1; -1 -1 -1]
    (stiffness)."""
    j = 3
    n = 2 ** j - 1
    h = 1.0 / 2 ** j
    med = space.Medium([1.0, 1.0], [1, 1], [1.0])
    M = space.mass(j, med).toarray()
    K = space.stiff(j, med).toarray()
    c = 3 * n + 3  # interior node (3,3)
    ms = np.array([[1, 4, 1], [4, 16, 4], [1, 4, 1]]) * h * h / 36
    ks = np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            assert abs(M[c, c + dy * n + dx] - ms[dy + 1, dx + 1]) < 1e-16
            assert abs(K[c, c + dy * n + dx] - ks[dy + 1, dx + 1]) < 1e-14


def test_dst_eigenpairs():
    """DST-I diagonalises the P1 matrices: q_k[i] = sin(i k pi/n),
    m_k = h/6 (4 + 2 cos(k pi/n)), kappa_k = 2/h (1 - cos(k pi/n))."""
    j, length = 5, 1.0
    n = 2 ** j
    h = length / n
    med = space.Medium([length], [1], [1.0])
    M = space.mass(j, med)
    K = space.stiff(j, med)
    i = np.arange(1, n)
    for k in (1, 7, n - 1):
        q = np.sin(i * k * np.pi / n)
        mk = h / 6 * (4 + 2 * np.cos(k * np.pi / n))
        kk = 2 / h * (1 - np.cos(k * np.pi / n))
        assert np.allclose(M @ q, mk * q, atol=1e-14)
        assert np.allclose(K @ q, kk * q, atol=1e-10)


def _brute_energy_1d(j, length, ncell, cv, u):
    """int c^2 (u_h')^2 on a sub-grid refining both the mesh and the blocks
    (u_h' and c are constant on each sub-interval: midpoint rule is exact)."""
    nsub = ncell * 2 ** 8   # refines the 2^j mesh (j <= 8) and the blocks
    xm = (np.arange(nsub) + 0.5) * length / nsub
    up = basis.hat_1d_deriv(j, length, xm) @ u
    cx = np.asarray(cv)[np.minimum((xm / (length / ncell)).astype(int), ncell - 1)]
    return np.sum(cx ** 2 * up ** 2) * length / nsub


def test_variable_speed_stiffness_energy_1d():
    """u^T K(c) u = int c^2 (u')^2, c piecewise constant and not aligned with
    the mesh (5 blocks on a 2^3 mesh)."""
    rng = np.random.default_rng(3)
    cv = rng.uniform(0.5, 2.0, 5)
    med = space.Medium([1.3], [5], cv)
    for j in (1, 3, 6):
        K = space.stiff(j, med)
        u = rng.standard_normal(2 ** j - 1)
        assert np.isclose(u @ (K @ u), _brute_energy_1d(j, 1.3, 5, cv, u), rtol=1e-12)


def test_variable_speed_stiffness_energy_2d():
    """u^T K(c) u = int c^2 |grad u|^2 in 2-D with 3x2 blocks not aligned with
    the level-2 mesh, by 2x2 Gauss on a sub-grid refining mesh and blocks."""
    rng = np.random.default_rng(4)
    ncx, ncy = 3, 2
    cv = rng.uniform(0.5, 2.0, ncx * ncy)
    lx, ly = 1.0, 0.8
    med = space.Medium([lx, ly], [ncx, ncy], cv)
    j = 2
    K = space.stiff(j, med)
    n = 2 ** j - 1
    u = rng.standard_normal(n * n)
    nsub = 2 ** j * ncx * ncy * 4
    g, gw = np.polynomial.legendre.leggauss(2)
    xs = ((np.arange(nsub)[:, None] + 0.5 + 0.5 * g[None, :]) * lx / nsub).reshape(-1)
    ys = ((np.arange(nsub)[:, None] + 0.5 + 0.5 * g[None, :]) * ly / nsub).reshape(-1)
    wx = np.tile(0.5 * gw, nsub) * lx / nsub
    wy = np.tile(0.5 * gw, nsub) * ly / nsub
    U = u.reshape(n, n)
    px, dpx = basis.hat_1d(j, lx, xs), basis.hat_1d_deriv(j, lx, xs)
    py, dpy = basis.hat_1d(j, ly, ys), basis.hat_1d_deriv(j, ly, ys)
    ux = py @ U @ dpx.T
    uy = dpy @ U @ px.T
    cx = np.minimum((xs / (lx / ncx)).astype(int), ncx - 1)
    cy = np.minimum((ys / (ly / ncy)).astype(int), ncy - 1)
    c2 = cv.reshape(ncy, ncx)[cy[:, None], cx[None, :]] ** 2
    brute = np.sum(wy[:, None] * wx[None, :] * c2 * (ux ** 2 + uy ** 2))
    assert np.isclose(u @ (K @ u), brute, rtol=1e-12)


def test_variable_speed_stiffness_partition_of_unity_1d():
    """The hats of the interior nodes sum to 1 away from the boundary, so every
    row of the exact K whose node is not next to the boundary sums to zero:
    hi + lo (the exact entries to ~32 digits) keeps this to ~1e-30 of the
    diagonal, block edges included (7 blocks not aligned with the mesh)."""
    from fractions import Fraction
    rng = np.random.default_rng(5)
    cv = rng.uniform(0.5, 2.0, 7)
    med = space.Medium([1.3], [7], cv)
    for j in (3, 6, 9):
        K = space.stiff(j, med).tocsr()
        Klo = space.stiff_lo(j, med).tocsr()
        assert np.array_equal(K.indices, Klo.indices)
        for r in range(1, 2 ** j - 2):
            a, b = K.indptr[r], K.indptr[r + 1]
            tot = sum(Fraction(float(x)) + Fraction(float(y))
                      for x, y in zip(K.data[a:b], Klo.data[a:b]))
            assert abs(float(tot)) <= 1e-30 * abs(K[r, r]), (j, r)
        # the rounded entries alone leave a last-bit row sum at block edges
        assert np.abs(Klo.data).max() <= 2.0 ** -52 * np.abs(K.data).max()


def test_cross_stiffness_galerkin_1d():
    """Phi^T K^J (exact entries) reproduces the coarse stiffness by nesting,
    Phi^T K^J Phi = K^a, agrees with the product of the separately built
    matrices, and vanishes at fine nodes inside a coarse element and a
    block (the coarse hat is linear there)."""
    rng = np.random.default_rng(6)
    cv = rng.uniform(0.5, 2.0, 8)
    med = space.Medium([1.0], [8], cv)
    J = 9
    KJ = space.stiff(J, med)
    for a in (1, 2, 4, 6):
        C = space.cross_stiff_1d(a, J, med)
        P = space.interp_1d(a, J, 1.0)
        ref = (P.T @ KJ).toarray()
        scale = np.abs(ref).max()
        assert np.abs(C.toarray() - ref).max() <= 1e-12 * scale
        Ka = space.stiff(a, med).toarray()
        assert np.abs((C @ P).toarray() - Ka).max() <= 1e-12 * np.abs(Ka).max()
        # nonzeros only at coarse nodes and block edges
        ratio, cell = 2 ** (J - a), 2 ** J // 8
        m = C.tocoo().col + 1
        assert np.all((m % ratio == 0) | (m % cell == 0))


def test_prolongation_nested():
    """Phi evaluates coarse hats at fine nodes, and composes: Phi_{a->J} =
    Phi_{a+1->J} Phi_{a->a+1} (nested P1 spaces)."""
    med = space.Medium([1.0], [1], [1.0])
    P = space.interp(2, 5, med).toarray()
    xs = np.arange(1, 32) / 32
    assert np.allclose(P, basis.hat_1d(2, 1.0, xs))
    P2 = space.interp(3, 5, med) @ space.interp(2, 3, med)
    assert np.allclose(P, P2.toarray())


# ------------------------------------------- component system (eqs. 6, 9) --

def _brute_bilinear(prob, jx, jt, nsub_t=32, nsub_x=2):
    """Dense matrix of the bilinear form (6) on V_jx (x) V_jt (1-D), by
    tensor Gauss quadrature of its three terms on a space-time sub-grid that
    refines the component mesh and the wave-speed blocks."""
    T = prob.T
    length = prob.medium.lengths[0]
    ncell = prob.medium.ncell[0]
    g, gw = np.polynomial.legendre.leggauss(4)
    nt = 2 ** jt * nsub_t
    nx = 2 ** jx * ncell * nsub_x
    tq = ((np.arange(nt)[:, None] + 0.5 + 0.5 * g) * T / nt).reshape(-1)
    tw = np.tile(0.5 * gw, nt) * T / nt
    xq = ((np.arange(nx)[:, None] + 0.5 + 0.5 * g) * length / nx).reshape(-1)
    xw = np.tile(0.5 * gw, nx) * length / nx
    ps = [basis.time_basis(jt, T, tq, k) for k in range(3)]
    dps0 = basis.time_basis(jt, T, np.array([0.0]), 1)[0]
    ph = basis.hat_1d(jx, length, xq)
    dph = basis.hat_1d_deriv(jx, length, xq)
    c = prob.medium.c.reshape(-1)[np.minimum((xq / (length / ncell)).astype(int), ncell - 1)]
    ew = tw * np.exp(-tq / T)
    nT, nX = ps[0].shape[1], ph.shape[1]
    S = np.zeros((nT * nX, nT * nX))
    for i in range(nT):
        for jj in range(nT):
            tt = np.sum(ew * ps[2][:, jj] * ps[1][:, i])      # (psi_j'', psi_i')_e
            t0 = dps0[jj] * dps0[i]                           # psi_j'(0) psi_i'(0)
            tb = np.sum(ew * ps[0][:, jj] * ps[1][:, i])      # (psi_j, psi_i')_e
            for k in range(nX):
                for l in range(nX):
                    mm = np.sum(xw * ph[:, l] * ph[:, k])
                    kk = np.sum(xw * c ** 2 * dph[:, l] * dph[:, k])
                    S[i * nX + k, jj * nX + l] = (tt + t0) * mm + tb * kk
    return S


def test_component_system_matches_bilinear_form_eq6():
    """S_c = A (x) M + B (x) K equals the Galerkin matrix of A(u,w), eq. (6),
    evaluated term by term by an independent space-time quadrature."""
    prob = Problem(1, [1.0], [3], [1.0, 0.6, 1.7], 1.3, 5)
    for jx, jt in [(2, 2), (1, 3), (3, 1)]:
        S = prob.system(jx, jt).toarray()   # high parts of A, B
        Sb = _brute_bilinear(prob, jx, jt)
        assert np.abs(S - Sb).max() <= 1e-12 * np.abs(Sb).max()
        # coercivity, eq. (8): symmetric part positive definite
        assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0


def test_load_matches_rhs_eq9():
    """b_c equals the right-hand side of eq. (9) for the interpolated nodal
    data, evaluated by an independent space-time quadrature."""
    rng = np.random.default_rng(11)
    prob = Problem(1, [1.0], [2], [1.0, 0.5], 1.0, 5)
    J, T = prob.J, prob.T
    nf = 2 ** J
    f = rng.standard_normal((nf + 1, nf - 1))
    u0 = rng.standard_normal(nf - 1)
    v0 = rng.standard_normal(nf - 1)
    g, gw = np.polynomial.legendre.leggauss(4)
    tq = ((np.arange(nf)[:, None] + 0.5 + 0.5 * g) * T / nf).reshape(-1)
    tw = np.tile(0.5 * gw, nf) * T / nf
    nx = nf * 2
    xq = ((np.arange(nx)[:, None] + 0.5 + 0.5 * g) * 1.0 / nx).reshape(-1)
    xw = np.tile(0.5 * gw, nx) / nx
    lam = basis.p1_time_hat(J, T, tq)                   # (tq, n)
    phJ = basis.hat_1d(J, 1.0, xq)
    dphJ = basis.hat_1d_deriv(J, 1.0, xq)
    F = lam @ f @ phJ.T                                  # interpolant at (t, x)
    c = np.where(xq < 0.5, 1.0, 0.5)
    for jx, jt in [(2, 3), (4, 1), (1, 4)]:
        dps = basis.time_basis(jt, T, tq, 1) * (tw * np.exp(-tq / T))[:, None]
        d0 = basis.time_basis(jt, T, np.array([0.0]), 1)[0]
        ph = basis.hat_1d(jx, 1.0, xq)
        dph = basis.hat_1d_deriv(jx, 1.0, xq)
        b = dps.T @ F @ (ph * xw[:, None])
        b += np.outer(d0, (phJ @ v0 * xw) @ ph)
        b -= np.outer(dps.sum(axis=0), (c ** 2 * (dphJ @ u0) * xw) @ dph)
        bo = prob.load(jx, jt, f, u0, v0)
        assert np.abs(bo - b).max() <= 1e-12 * np.abs(b).max()


def test_structured_solve_equals_dense_lu():
    """The refined sparse solve equals a dense LU solve of the explicit S_c."""
    rng = np.random.default_rng(5)
    prob = Problem(2, [1.0, 1.0], [2, 2], [1.0, 0.7, 1.4, 0.9], 1.0, 5)
    for jx, jt in [(2, 2), (1, 3), (3, 1)]:
        S = prob.system(jx, jt).toarray()
        b = rng.standard_normal(S.shape[0]).reshape(2 ** jt + 1, -1)
        x = prob.solve(jx, jt, b)
        xd = np.linalg.solve(S, b.reshape(-1))
        assert np.abs(x.reshape(-1) - xd).max() <= 1e-12 * np.abs(xd).max()
        xt = prob.solve(jx, jt, b, transpose=True)
        xdt = np.linalg.solve(S.T, b.reshape(-1))
        assert np.abs(xt.reshape(-1) - xdt).max() <= 1e-12 * np.abs(xdt).max()


# -------------------------------------------------------- rates (eqs. 14, 18, Thm 1)

def _rate(errs):
    return [math.log2(a / b) for a, b in zip(errs[:-1], errs[1:])]


def test_time_only_ode_rate_eq14():
    """Prop. 1 (spatial eigenbasis): with one spatial mode the time problem is
    the Galerkin form of u'' + mu u = 0, u(0) = 0, u'(0) = 1.  Quadratic C^1
    splines converge at O(h_t^3) in L^2 (eq. 14 with p_t = 2)."""
    mu, T = 12.0, 1.0
    errs = []
    for jt in range(3, 9):
        tm = timemat.time_matrices(jt, T)
        u = np.linalg.solve(tm["A"] + mu * tm["B"], tm["d0"] * 1.0)
        tq, tw = method.fine_quadrature(jt + 1, T)
        uh = basis.time_basis(jt, T, tq) @ u
        ue = np.sin(math.sqrt(mu) * tq) / math.sqrt(mu)
        errs.append(math.sqrt(np.sum(tw * (uh - ue) ** 2)))
    rates = _rate(errs)
    assert all(2.7 < r < 3.3 for r in rates[-3:]), rates


_OM = 5 * math.pi / 4


def _s(t):
    return t ** 6 * np.sin(_OM * t) ** 2


def _s2(t):
    q = np.sin(_OM * t) ** 2
    q1 = _OM * np.sin(2 * _OM * t)
    q2 = 2 * _OM ** 2 * np.cos(2 * _OM * t)
    return 30 * t ** 4 * q + 12 * t ** 5 * q1 + t ** 6 * q2


def _manufactured_1d():
    """Sec. 6.1 solution moved to (0,1): u = t^6 sin(pi x) sin^2(5 pi t/4),
    c = 1, u0 = v0 = 0, f = u_tt - u_xx (compatible data, eqs. 24-25)."""
    u = lambda t, x: _s(t) * np.sin(np.pi * x)
    f = lambda t, x: (_s2(t) + np.pi ** 2 * _s(t)) * np.sin(np.pi * x)
    z = lambda x: 0.0 * x
    gz = lambda x: (0.0 * x,)
    return u, f, z, z, gz


@pytest.mark.parametrize("load_kind", ["exact", "nodal"])
def test_sparse_and_full_grid_rates_1d(load_kind):
    """Eq. (18) and Theorem 1 with (p_x, p_t) = (1, 2): full-grid and
    sparse-grid L^2(Q_T) errors both decay as 2^{-2J} (no log factor since
    p_x != p_t).  'nodal' feeds the finest-grid nodal values through the
    library's load (an O(h^2) interpolation of the data)."""
    u, f, u0, v0, gu0 = _manufactured_1d()
    es, ef = [], []
    for L in range(6, 11):
        prob = Problem(1, [1.0], [1], [1.0], 1.0, L)
        J = prob.J
        if load_kind == "exact":
            ld = lambda jx, jt: method.load_exact(prob, jx, jt, f, u0, v0, gu0)
        else:
            tn = np.arange(2 ** J + 1) / 2 ** J
            xn = np.arange(1, 2 ** J) / 2 ** J
            fn = f(tn[:, None], xn[None, :])
            zz = np.zeros(2 ** J - 1)
            ld = lambda jx, jt: prob.load(jx, jt, fn, zz, zz)
        sols = [prob.solve(jx, jt, ld(jx, jt)) for jx, jt, _ in prob.comps]
        e, nrm = method.l2_error(prob, sols, u)
        es.append(e / nrm)
        fg = [prob.solve(J, J, ld(J, J))]
        e, nrm = method.l2_error(prob, fg, u, comps=[(J, J, 1)])
        ef.append(e / nrm)
    rs, rf = _rate(es), _rate(ef)
    assert all(1.9 < r < 2.15 for r in rs[-2:]), (es, rs)
    # the full grid approaches slope 2 (from above with the exact load)
    assert 1.9 < rf[-1] < 2.15 and abs(rf[-1] - 2) <= abs(rf[-2] - 2), (ef, rf)
    # Sec. 6.1 / eq. (26a): for a comparable number of unknowns the sparse
    # grid is more accurate.  Compare sparse L=10 with the largest full grid
    # that has no more unknowns than it.
    ns = levels.n_sparse(10, 1)
    fulls = [(levels.n_space(L - 1, 1) * levels.n_time(L - 1), e)
             for L, e in zip(range(6, 11), ef)]
    n_f, e_f = max((nf, e) for nf, e in fulls if nf <= ns)
    assert es[-1] < e_f, (ns, n_f, es[-1], e_f)


def test_sparse_grid_rate_2d():
    """Theorem 1 in 2+1 dimensions (Q1 x quadratic C^1):
    u = t^6 sin(pi x) sin(pi y) sin^2(5 pi t/4), c = 1, compatible data."""
    u = lambda t, x, y: _s(t) * np.sin(np.pi * x) * np.sin(np.pi * y)
    f = lambda t, x, y: (_s2(t) + 2 * np.pi ** 2 * _s(t)) * np.sin(np.pi * x) * np.sin(np.pi * y)
    z = lambda x, y: 0.0 * x * y
    gz = lambda x, y: (0.0 * x * y, 0.0 * x * y)
    errs = []
    for L in range(4, 8):
        prob = Problem(2, [1.0, 1.0], [1, 1], [1.0], 1.0, L)
        sols = [prob.solve(jx, jt, method.load_exact(prob, jx, jt, f, z, z, gz))
                for jx, jt, _ in prob.comps]
        e, nrm = method.l2_error(prob, sols, u)
        errs.append(e / nrm)
    r = _rate(errs)
    assert 1.7 < r[-1] < 2.4, (errs, r)


# ------------------------------------------------ combination formula ------

def _all_projections(prob, f, u0, v0):
    """P_{jx,jt} u for every level pair 1..L-1 (each the Galerkin solve)."""
    P = {}
    for jx in range(1, prob.L):
        for jt in range(1, prob.L):
            P[(jx, jt)] = prob.solve(jx, jt, prob.load(jx, jt, f, u0, v0))
    return P


def test_combination_equals_detail_sum_eq21():
    """Eq. (19) equals the sum of the details Delta^P (eq. 20) over
    jx'+jt' <= J (eq. 21), and P_{J,J} - u^CF is the sum over the rest
    (eq. 21bis); details are formed on the finest grid."""
    rng = np.random.default_rng(7)
    prob = Problem(1, [1.0], [2], [1.0, 0.6], 1.0, 5)
    nf = 2 ** prob.J
    f = rng.standard_normal((nf + 1, nf - 1))
    u0 = rng.standard_normal(nf - 1)
    v0 = rng.standard_normal(nf - 1)
    P = _all_projections(prob, f, u0, v0)
    Pf = {k: prob.prolong(k[0], k[1], v) for k, v in P.items()}
    zero = np.zeros((nf + 1, nf - 1))
    get = lambda a, b: Pf.get((a, b), zero)  # level 0 (paper's -1) is zero

    def delta(a, b):
        return get(a, b) - get(a - 1, b) - get(a, b - 1) + get(a - 1, b - 1)

    ucf = prob.combine(prob.component_solutions(f, u0, v0), np.zeros(nf - 1))
    Jp = prob.L - 2   # paper's J; paper level j' = our level - 1
    dsum = sum(delta(a, b) for a in range(1, prob.L) for b in range(1, prob.L)
               if (a - 1) + (b - 1) <= Jp)
    assert np.abs(ucf - dsum).max() < 1e-10 * np.abs(ucf).max()
    rest = sum(delta(a, b) for a in range(1, prob.L) for b in range(1, prob.L)
               if (a - 1) + (b - 1) > Jp)
    pjj = Pf[(prob.L - 1, prob.L - 1)]
    assert np.abs((pjj - ucf) - rest).max() < 1e-10 * np.abs(pjj).max()


def _l2e_projection_coeffs(jt, T, g_fn):
    """Coefficients of the L^2_e(0,T)-orthogonal projection of g onto V_jt."""
    tq, tw = method.fine_quadrature(jt + 3, T)
    P = basis.time_basis(jt, T, tq)
    w = tw * np.exp(-tq / T)
    G = P.T @ (P * w[:, None])
    return np.linalg.solve(G, P.T @ (w * g_fn(tq)))


def test_projector_combination_exact_on_sparse_space():
    """Classical combination-technique identity for nested commuting
    projectors (nodal interpolation in x, L^2_e projection in t): feeding the
    components (I_jx (x) Q_jt) g, the signed combination of eq. (19) returns g
    exactly iff g lies in the sparse space sum_{c} V_jx (x) V_jt, and not for a
    generic full-grid g."""
    T = 1.0
    prob = Problem(1, [1.0], [1], [1.0], T, 5)
    rng = np.random.default_rng(2)
    terms = []  # g = sum of products phi(x) w(t), each in some V_a (x) V_{L-a}
    for a in range(1, prob.L):
        cx = rng.standard_normal(2 ** a - 1)
        ct = rng.standard_normal(2 ** (prob.L - a) + 1)
        terms.append((a, prob.L - a, cx, ct))

    def run(terms):
        nf = 2 ** prob.J
        xn = np.arange(1, nf) / nf
        tn = np.arange(nf + 1) / nf
        exact = 0.0
        for a, b, cx, ct in terms:
            exact = exact + np.outer(basis.time_basis(b, T, tn) @ ct,
                                     basis.hat_1d(a, 1.0, xn) @ cx)
        sols = []
        for jx, jt, _ in prob.comps:
            u = 0.0
            for a, b, cx, ct in terms:
                gx = basis.hat_1d(a, 1.0, np.arange(1, 2 ** jx) / 2 ** jx) @ cx
                qt = _l2e_projection_coeffs(jt, T, lambda t: basis.time_basis(b, T, t) @ ct)
                u = u + np.outer(qt, gx)
            sols.append(u)
        return prob.combine(sols, np.zeros(nf - 1)), exact

    got, exact = run(terms)
    assert np.abs(got - exact).max() <= 1e-12 * np.abs(exact).max()
    # a function of the full finest grid is not reproduced
    J = prob.J
    full = [(J, J, rng.standard_normal(2 ** J - 1), rng.standard_normal(2 ** J + 1))]
    got, exact = run(full)
    assert np.abs(got - exact).max() > 1e-2 * np.abs(exact).max()


def test_coarsest_space_reproduced():
    """If the load of every component is A(u*, .) for u* in V_1 (x) V_1 (a
    subspace of every component space), each Galerkin solve returns u*
    (eq. 10 projector property) and the combination returns u* (sum of
    signs = 1)."""
    T = 1.0
    prob = Problem(1, [1.0], [2], [1.0, 0.5], T, 6)
    rng = np.random.default_rng(9)
    cx = rng.standard_normal(1)
    ct = rng.standard_normal(3)
    sols = []
    for jx, jt, _ in prob.comps:
        gx = basis.hat_1d(1, 1.0, np.arange(1, 2 ** jx) / 2 ** jx) @ cx
        # u* restricted to V_jt: exact coefficients by interpolation at
        # enough points (nested spaces => exact)
        tq = np.linspace(0, T, 4 * 2 ** jt + 7)
        Pt = basis.time_basis(jt, T, tq)
        gt = np.linalg.lstsq(Pt, basis.time_basis(1, T, tq) @ ct, rcond=None)[0]
        ustar = np.outer(gt, gx)
        b = (prob.system(jx, jt) @ ustar.reshape(-1)).reshape(ustar.shape)
        sols.append(prob.solve(jx, jt, b))
        assert np.abs(sols[-1] - ustar).max() < 1e-10
    nf = 2 ** prob.J
    U = prob.combine(sols, np.zeros(nf - 1))
    tn = np.arange(nf + 1) / nf
    xn = np.arange(1, nf) / nf
    ex = np.outer(basis.time_basis(1, T, tn) @ ct, basis.hat_1d(1, 1.0, xn) @ cx)
    assert np.abs(U - ex).max() < 1e-10


# ------------------------------------------------------------- adjoint -----

@pytest.mark.parametrize("d", [1, 2])
def test_adjoint_dot_product_and_dense(d):
    """<F x, g> = <x, F^T g>; for a tiny level the adjoint equals the
    transpose of the forward map assembled column by column."""
    rng = np.random.default_rng(13)
    if d == 1:
        prob = Problem(1, [1.0], [3], [1.0, 1.5, 0.7], 1.2, 4)
    else:
        prob = Problem(2, [1.0, 0.9], [2, 2], [1.0, 1.5, 0.7, 1.1], 1.0, 3)
    nt, ns = prob.nt_fine, prob.ns_fine
    f = rng.standard_normal((nt, ns))
    u0 = rng.standard_normal(ns)
    v0 = rng.standard_normal(ns)
    g = rng.standard_normal((nt, ns))
    U = prob.forward(f, u0, v0)
    df, du0, dv0 = prob.adjoint(g)
    lhs = np.sum(U * g)
    rhs = np.sum(f * df) + u0 @ du0 + v0 @ dv0
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # dense transpose
    n_in = nt * ns + 2 * ns
    F = np.zeros((nt * ns, n_in))
    for k in range(n_in):
        e = np.zeros(n_in)
        e[k] = 1.0
        F[:, k] = prob.forward(e[:nt * ns].reshape(nt, ns), e[nt * ns:nt * ns + ns],
                               e[nt * ns + ns:]).reshape(-1)
    adj = np.concatenate([df.reshape(-1), du0, dv0])
    assert np.abs(F.T @ g.reshape(-1) - adj).max() <= 1e-11 * np.abs(adj).max()


def test_gradient_central_differences():
    """Least-squares loss 1/2 ||U - U_obs||^2: the adjoint gradient agrees with
    central differences (the loss is quadratic, so only roundoff remains)."""
    rng = np.random.default_rng(17)
    prob = Problem(1, [1.0], [4], [1.0, 0.6, 1.8, 1.2], 1.0, 5)
    nt, ns = prob.nt_fine, prob.ns_fine
    f = rng.standard_normal((nt, ns))
    u0 = rng.standard_normal(ns)
    v0 = np.zeros(ns)
    Uobs = rng.standard_normal((nt, ns))
    loss = lambda f_, u0_: 0.5 * np.sum((prob.forward(f_, u0_, v0) - Uobs) ** 2)
    df, du0, _ = prob.adjoint(prob.forward(f, u0, v0) - Uobs)
    h = 1e-6
    for _ in range(4):
        pf = rng.standard_normal((nt, ns))
        pu = rng.standard_normal(ns)
        nrm = math.sqrt(np.sum(pf ** 2) + np.sum(pu ** 2))
        pf, pu = pf / nrm, pu / nrm
        fd = (loss(f + h * pf, u0 + h * pu) - loss(f - h * pf, u0 - h * pu)) / (2 * h)
        ad = np.sum(df * pf) + du0 @ pu
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-6


# ---- energy of the computed solution (Sec. 6.3) -----------------------------

def _single_coefficient(prob, jx, jt, i, k):
    """Component solutions that are zero except u_(jx,jt)[i, k] = 1."""
    sols = []
    for cx, ct, _ in prob.comps:
        u = np.zeros((levels.n_time(ct), levels.n_space(cx, prob.d)))
        if (cx, ct) == (jx, jt):
            u[i, k] = 1.0
        sols.append(u)
    return sols


def test_energy_single_basis_function_closed_form():
    """u_h = psi_i(t) phi_k(x) with an interior uniform quadratic B-spline psi_i
    (knot spacing tau) and an interior level-a hat (width h): E(t) =
    1/2 psi_i'(t)^2 (2h/3) + 1/2 psi_i(t)^2 (2 c^2/h).  At the middle of the
    spline's central interval psi = 3/4, psi' = 0; at its second knot psi = 1/2,
    psi' = 1/tau."""
    prob = Problem(1, [1.0], [1], [1.3], 1.0, 6)            # J = 5
    jx, jt, i, k = 2, 4, 5, 1                                # h = 1/4, tau = 1/16
    assert (jx, jt, 1) in prob.comps
    sols = _single_coefficient(prob, jx, jt, i, k)
    h, tau, c2 = 0.25, 1.0 / 16, 1.3 ** 2
    # psi_5 = B_6: support [4 tau, 7 tau]
    E = method.energy(prob, sols, np.zeros(prob.ns_fine), [5.5 * tau, 5.0 * tau])
    want = [0.5 * (3 / 4) ** 2 * 2 * c2 / h,
            0.5 * (1 / tau) ** 2 * 2 * h / 3 + 0.5 * (1 / 2) ** 2 * 2 * c2 / h]
    np.testing.assert_allclose(E, want, rtol=1e-13)


def test_energy_single_basis_function_closed_form_2d():
    """2-D: phi_k = hat_x hat_y, int phi^2 = (2h/3)^2, int |grad phi|^2 =
    2 (2/h)(2h/3) (c = 1), at the middle of the spline's central interval."""
    prob = Problem(2, [1.0, 1.0], [1, 1], [1.0], 1.0, 6)
    jx, jt, i = 2, 4, 5
    k = 1 * 3 + 1                                            # centre node of level 2
    sols = _single_coefficient(prob, jx, jt, i, k)
    h, tau = 0.25, 1.0 / 16
    E = method.energy(prob, sols, np.zeros(prob.ns_fine), [5.5 * tau])
    want = 0.5 * (3 / 4) ** 2 * 2 * (2 / h) * (2 * h / 3)
    np.testing.assert_allclose(E, [want], rtol=1e-13)


def test_solution_at_nodes_equals_combination():
    """At the finest time nodes the arbitrary-instant evaluation reproduces
    the nodal combination U (eq. 19 plus the lift)."""
    prob = Problem(1, [1.0], [2], [1.0, 0.6], 1.0, 5)
    rng = np.random.default_rng(3)
    sols = [rng.standard_normal((levels.n_time(jt), levels.n_space(jx, 1)))
            for jx, jt, _ in prob.comps]
    u0 = rng.standard_normal(prob.ns_fine)
    t = np.arange(prob.nt_fine) * prob.T / 2 ** prob.J
    np.testing.assert_allclose(method.solution_at(prob, sols, u0, t),
                               prob.combine(sols, u0), rtol=0, atol=1e-12)


def test_solution_time_derivative_by_central_difference():
    """d_t u_h is a quadratic polynomial in t inside every finest interval, so
    a central difference inside one interval reproduces it to rounding."""
    prob = Problem(2, [1.0, 1.0], [1, 1], [1.0], 1.0, 4)
    rng = np.random.default_rng(4)
    sols = [rng.standard_normal((levels.n_time(jt), levels.n_space(jx, 2)))
            for jx, jt, _ in prob.comps]
    u0 = np.zeros(prob.ns_fine)
    dt = prob.T / 2 ** prob.J
    t = np.array([0.3, 2.5, 5.7]) * dt                       # inside intervals
    d = 0.2 * dt
    fd = (method.solution_at(prob, sols, u0, t + d) -
          method.solution_at(prob, sols, u0, t - d)) / (2 * d)
    np.testing.assert_allclose(method.solution_at(prob, sols, u0, t, deriv=1), fd,
                               rtol=0, atol=1e-9 * np.abs(fd).max())


def test_energy_converges_to_the_exact_energy():
    """f = 0, u0 = 0, v0 = pi sin(pi x), c = 1: u = sin(pi t) sin(pi x) keeps
    E = pi^2/4; the sparse-grid energy approaches it as L grows."""
    errs = []
    for L in (5, 6, 7):
        prob = Problem(1, [1.0], [1], [1.0], 1.0, L)
        x = np.arange(1, 2 ** prob.J) / 2 ** prob.J
        f = np.zeros((prob.nt_fine, prob.ns_fine))
        u0 = np.zeros(prob.ns_fine)
        v0 = np.pi * np.sin(np.pi * x)
        sols = prob.component_solutions(f, u0, v0)
        E = method.energy(prob, sols, u0, [0.25, 0.5, 0.75])
        errs.append(np.abs(E / (np.pi ** 2 / 4) - 1).max())
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-2
