"""CPU tests of the HIP library's host side: exported symbols and the tables
it builds, checked against the oracle (no device calls)."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import timemat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgwave.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2606_09688_amd as sg
    L = ctypes.CDLL(sg.LIB_PATH)
    names = _declared()
    assert "sg_assemble" in names and "sg_adjoint" in names
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("b,T", [(1, 1.0), (2, 1.0), (4, 2.0), (7, 0.5)])
def test_host_time_matrices_match_oracle(b, T):
    """Banded A_b, B_b (Prop. 1), derivative values and g of the library's
    host code equal the oracle's independent Cox-de Boor / quadrature ones."""
    import paper_2606_09688_amd as sg
    h = sg.host_time_level(b, T)
    Dlo, Dhi, g = h["Dlo"], h["Dhi"], h["g"]
    tm = timemat.time_matrices(b, T)
    dd = timemat.time_matrices_dd(b, T)
    n = 2 ** b + 1
    for name in ("A", "B"):
        # double-double entries agree with the oracle's 40-digit ones
        diff = (h[name] - dd[name + "_hi"]) + (h[name + "lo"] - dd[name + "_lo"])
        assert np.abs(diff).max() <= 1e-29 * np.abs(dd[name + "_hi"]).max(), name
    assert np.allclose(g, tm["g"], rtol=1e-14, atol=1e-15)
    # psi_i'(t_q) at the level-b nodes from the oracle's basis derivatives
    from oracle import basis
    tq = T * np.arange(n) / 2 ** b
    dpsi = basis.time_basis(b, T, np.clip(tq, 0, T), 1)  # (q, i)
    for i in range(n):
        assert abs(Dlo[i] - dpsi[i, i]) <= 1e-12 * abs(dpsi).max()
        if i + 1 < n:
            assert abs(Dhi[i] - dpsi[i + 1, i]) <= 1e-12 * abs(dpsi).max()
    assert tm["d0"][0] == pytest.approx(Dlo[0], rel=1e-14)


def _dense_taps(q0, w, nq):
    n = len(q0)
    M = np.zeros((nq, n))
    for k in range(n):
        for o in range(3):
            if w[k, o] != 0:
                M[q0[k] + o, k] += w[k, o]
    return M


@pytest.mark.parametrize("b,J,T", [(1, 3, 1.0), (2, 5, 1.0), (3, 3, 2.0), (4, 7, 0.8)])
def test_host_taps_compose_to_oracle_load_and_evaluation(b, J, T):
    """P1 taps followed by the derivative values D_b reproduce the oracle's
    load factor W (eq. 9 with P1-in-time data); spline taps equal the
    oracle's basis values at the fine nodes; the windows are monotone with
    unit steps as the streaming kernels assume."""
    import paper_2606_09688_amd as sg
    nq = 2 ** b + 1
    q0, w = sg.host_taps(0, b, J, T)
    assert np.all(np.diff(q0) >= 0) and np.all(np.diff(q0) <= 1)
    assert q0.min() >= 0 and q0.max() <= nq - 3
    P1 = _dense_taps(q0, w, nq)                     # (q, n)
    h = sg.host_time_level(b, T)
    D = np.diag(h["Dlo"]) + np.diag(h["Dhi"][:-1], 1)         # D[i, q] nonzero at q = i, i+1
    W = timemat.load_weights(b, J, T)
    assert np.abs(D @ P1 - W).max() <= 1e-13 * np.abs(W).max()
    q0s, ws = sg.host_taps(1, b, J, T)
    assert np.all(np.diff(q0s) >= 0) and np.all(np.diff(q0s) <= 1)
    Psi = _dense_taps(q0s, ws, nq).T                # (n, i)
    assert np.abs(Psi - timemat.eval_at_nodes(b, J, T)).max() <= 1e-15


@pytest.mark.parametrize("a,length,cv", [(1, 1.0, [0.8]), (3, 1.0, [1.0, 0.5]),
                                         (5, 2.0, [0.5, 2.0, 1.3, 0.7]),
                                         (6, 1.0, list(np.linspace(0.5, 2.0, 8))),
                                         (8, 1.0, [1.0, 0.5])])
def test_host_pencil_eigenpairs_of_oracle_matrices(a, length, cv):
    """The variable-speed modes (1-D) are the generalised eigenpairs of the
    oracle's own P1 matrices: K V = M V diag(lam), V^T M V = I (eq. (9),
    spatial matrices with c^2 integrated exactly over each element)."""
    import paper_2606_09688_amd as sg
    from oracle.space import Medium, mass, stiff
    med = Medium([length], [len(cv)], cv)
    M = mass(a, med).toarray()
    K = stiff(a, med).toarray()
    V, lam = sg.host_pencil(a, length, cv)
    n = 2 ** a - 1
    assert V.shape == (n, n)
    scale = np.abs(K).max()
    assert np.abs(K @ V - M @ V * lam[None, :]).max() <= 1e-13 * scale * max(1.0, np.abs(V).max())
    assert np.abs(V.T @ M @ V - np.eye(n)).max() <= 1e-13
    # the eigenvalues are those of the pencil (dense reference for small n)
    ref = np.sort(np.linalg.eigvals(np.linalg.solve(M, K)).real)
    assert np.allclose(np.sort(lam), ref, rtol=1e-10, atol=0)


@pytest.mark.parametrize("a,lengths,ncell", [(2, [1.0, 1.0], [4, 4]), (3, [1.0, 1.0], [4, 4]),
                                              (3, [1.0, 0.8], [3, 2]), (4, [1.3, 1.0], [4, 4])])
def test_host_pencil_2d_matches_oracle_matrices(a, lengths, ncell):
    """The dense 2-D variable-speed pencil the library diagonalises (rocSOLVER,
    at assembly) is the oracle's Q1 mass and stiffness of eq. (9), blocks
    aligned with the mesh or not."""
    import paper_2606_09688_amd as sg
    from oracle.space import Medium, mass, stiff
    rng = np.random.default_rng(10 + a)
    cv = rng.uniform(0.5, 2.0, ncell[0] * ncell[1])
    med = Medium(lengths, ncell, cv)
    K_ref = stiff(a, med).toarray()
    M_ref = mass(a, med).toarray()
    K, M = sg.host_pencil_2d(a, lengths, ncell, cv)
    assert np.array_equal(K, K.T) and np.array_equal(M, M.T)
    assert np.abs(K - K_ref).max() <= 1e-13 * np.abs(K_ref).max()
    assert np.abs(M - M_ref).max() <= 1e-13 * np.abs(M_ref).max()
    # a pencil with a sign or a block slip is not symmetric positive definite
    # with the oracle's spectrum
    lam = np.sort(np.linalg.eigvals(np.linalg.solve(M, K)).real)
    ref = np.sort(np.linalg.eigvals(np.linalg.solve(M_ref, K_ref)).real)
    assert np.allclose(lam, ref, rtol=1e-10, atol=0) and lam[0] > 0


def test_mass_of_level1_interpolant_is_fixed_stencil():
    """The 2-D df prolongation never forms the fine field: per axis, the fine
    P1 mass matrix applied to the interpolant of level J-1 values z is
    h/12 (z_{K-1} + 10 z_K + z_{K+1}) at fine node 2K and h/2 (z_K + z_{K+1})
    at 2K+1 (checked on the oracle's own matrices, boundary values zero)."""
    from oracle.space import interp_1d, mass_1d
    J, length = 6, 1.3
    h = length / 2 ** J
    MJ = mass_1d(J, length).toarray()
    Phi = interp_1d(J - 1, J, length).toarray()
    z = np.random.default_rng(7).standard_normal(2 ** (J - 1) - 1)
    ref = MJ @ Phi @ z
    zp = np.concatenate([[0.0], z, [0.0]])   # level J-1 nodes 0 .. 2^(J-1)
    got = np.empty(2 ** J - 1)
    for m in range(1, 2 ** J):
        K = m // 2
        if m % 2 == 0:
            got[m - 1] = h / 12 * (zp[K - 1] + 10 * zp[K] + zp[K + 1])
        else:
            got[m - 1] = h / 2 * (zp[K] + zp[K + 1])
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("b,T", [(1, 1.0), (2, 1.0), (3, 1.0), (3, 0.7), (4, 1.0), (5, 2.0)])
def test_host_time_diagonalisation_solves_oracle_systems(b, T):
    """The time diagonalisation used for the 2-D variable-speed components
    (B^{-1} A = V diag(lam) V^{-1}, Prop. 1 time matrices): with a scalar
    spatial pair (M, K) = (1, mu) the component system is A + mu B, and its
    solution (and that of the transpose) assembled from the returned tables
    equals a dense solve with the oracle's exact time matrices.  The unique
    eigenvalues are the oracle's spectrum, one of each conjugate pair."""
    import paper_2606_09688_amd as sg
    dd = timemat.time_matrices_dd(b, T)
    A = timemat.band_to_dense(dd["A_hi"]) + timemat.band_to_dense(dd["A_lo"])
    B = timemat.band_to_dense(dd["B_hi"]) + timemat.band_to_dense(dd["B_lo"])
    h = sg.host_time_fdm(b, T)
    lam = h["lam"]
    nq = 2 ** b + 1
    ref = np.linalg.eigvals(np.linalg.solve(B, A))
    full = np.concatenate([lam, np.conj(lam[np.abs(lam.imag) > 0])])
    assert full.size == nq
    key = lambda z: (round(z.real, 6), round(z.imag, 6))
    assert np.allclose(sorted(full, key=key), sorted(ref, key=key), rtol=1e-10)
    assert np.all(lam.imag >= 0)
    rng = np.random.default_rng(b)
    for mu in (0.0, 3.7, 250.0, 1e5):
        rhs = rng.standard_normal(nq)
        S = A + mu * B
        x_ref = np.linalg.solve(S, rhs)
        x = np.real(h["fout"] @ ((h["fin"] @ rhs) / (lam + mu)))
        assert np.abs(x - x_ref).max() <= 1e-12 * np.abs(x_ref).max(), mu
        z_ref = np.linalg.solve(S.T, rhs)
        z = np.real(h["aout"] @ ((h["ain"] @ rhs) / (lam + mu)))
        assert np.abs(z - z_ref).max() <= 1e-12 * np.abs(z_ref).max(), mu


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("b, J, chunk", [(1, 9, 176), (2, 9, 176), (3, 9, 176), (2, 5, 8),
                                         (4, 6, 64), (5, 5, 8), (2, 12, 1368)])
def test_time_chunks_hold_the_finest_window_fixed(kind, b, J, chunk):
    """The chunks a streaming pass takes when the finest level's component has
    time level b (a coarsest level b of the combination): they tile the slabs
    0..2^J in order, none is empty, q0 is constant on each (the kernels keep
    the finest level's three coefficients fixed per block), and the chunk
    length is the longest such one up to the requested length (for b = 1,
    the requested length with no phase)."""
    import paper_2606_09688_amd as sg
    q0, _ = sg.host_taps(kind, b, J, 1.0)
    ntf = 2 ** J + 1
    c, ph, nch = sg.host_time_chunks(q0, chunk)
    assert 1 <= c <= chunk and 0 <= ph < c
    spans = [(max(0, k * c - ph), min((k + 1) * c - ph, ntf)) for k in range(nch)]
    assert spans[0][0] == 0 and spans[-1][1] == ntf
    assert all(a < e for a, e in spans)
    assert all(spans[k][1] == spans[k + 1][0] for k in range(nch - 1))
    for a, e in spans:
        assert np.all(q0[a:e] == q0[a])
    if b == 1:
        assert (c, ph) == (chunk, 0)
    # no longer chunk length would do
    moves = [n for n in range(1, ntf) if q0[n] != q0[n - 1]]
    for c2 in range(c + 1, chunk + 1):
        p2 = (c2 - moves[0] % c2) % c2
        assert any((n + p2) % c2 for n in moves)
