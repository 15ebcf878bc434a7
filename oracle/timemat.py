"""Time matrices and time load factors (oracle; test infrastructure).

Paper, proof of Prop. 1 (eq. 30): with a basis {psi_i} of V^t_{jt},

    A[i,j] = (psi_j'', psi_i')_{L^2_e(0,T)} + psi_j'(0) psi_i'(0),
    B[i,j] = (psi_j,   psi_i')_{L^2_e(0,T)},

where (u,v)_{L^2_e} = int_0^T u v e^{-t/T} dt (Notation section).  The
right-hand side of eq. (9) contributes, per time test function psi_i,

    (f, psi_i')_{L^2_e},   psi_i'(0) (v0, .),   -(int_0^T psi_i' e^{-t/T} dt) (c^2 grad u0, grad .).

Nodal data reading (the paper integrates exact data): the library receives f
as values at the finest time nodes t_n = n T/2^J (n = 0..2^J) and uses its
piecewise-linear interpolant in t, so the time factor of the f-term is

    W[i,n] = int_0^T lambda_n(t) psi_i'(t) e^{-t/T} dt,

lambda_n the P1 hat of t_n.  All integrals: 8-point Gauss-Legendre per
element of the relevant mesh (level jt for A, B, M_e, K_e, g; the finest
level J for W, on which psi_i is polynomial).  The integrands are
polynomials of degree <= 3 times e^{-t/T}; the rule error is far below
double-precision roundoff.

Also returned for the identity checks of eqs. (2)-(3):
M_e[i,j] = (psi_j, psi_i)_{L^2_e}, K_e[i,j] = (psi_j', psi_i')_{L^2_e},
d0 = psi'(0), dT = psi'(T), eT = psi(T).
"""

import numpy as np

from . import basis

_NQ = 8
_GX, _GW = np.polynomial.legendre.leggauss(_NQ)


def _elem_points(a, b):
    return 0.5 * (b - a) * _GX + 0.5 * (a + b), 0.5 * (b - a) * _GW


def _knots(jt, T):
    key = (jt, float(T))
    if key not in _KNOT_CACHE:
        _KNOT_CACHE[key] = basis.clamped_knots(jt, T)
    return _KNOT_CACHE[key]


_KNOT_CACHE = {}


def _span_values(jt, T, e, t, deriv):
    """psi_i^{(deriv)} on element e of level jt: returns (indices, values).

    Element e = [e h, (e+1) h] is knot span s = e + 2; the nonzero B-splines
    there are B_e, B_{e+1}, B_{e+2}, i.e. psi_{e-1}, psi_e, psi_{e+1}
    (psi_{-1} = B_0 is the dropped function)."""
    knots = _knots(jt, T)
    vals = basis.local_basis(knots, 2, e + 2, t, deriv)
    idx = [e - 1, e, e + 1]
    keep = [k for k in range(3) if idx[k] >= 0]
    return [idx[k] for k in keep], vals[:, keep]


def time_matrices(jt, T):
    """Dictionary with A, B, M_e, K_e (dense), g, d0, dT, eT at level jt."""
    N = 2 ** jt
    h = T / N
    n = N + 1
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    Me = np.zeros((n, n))
    Ke = np.zeros((n, n))
    g = np.zeros(n)
    for e in range(N):
        tq, wq = _elem_points(e * h, (e + 1) * h)
        w = wq * np.exp(-tq / T)
        idx, v0 = _span_values(jt, T, e, tq, 0)
        _, v1 = _span_values(jt, T, e, tq, 1)
        _, v2 = _span_values(jt, T, e, tq, 2)
        for a, i in enumerate(idx):
            g[i] += np.sum(w * v1[:, a])
            for b, j in enumerate(idx):
                A[i, j] += np.sum(w * v2[:, b] * v1[:, a])
                B[i, j] += np.sum(w * v0[:, b] * v1[:, a])
                Me[i, j] += np.sum(w * v0[:, b] * v0[:, a])
                Ke[i, j] += np.sum(w * v1[:, b] * v1[:, a])
    d0 = np.zeros(n)
    idx, v = _span_values(jt, T, 0, np.array([0.0]), 1)
    d0[idx] = v[0]
    dT = np.zeros(n)
    eT = np.zeros(n)
    idx, v = _span_values(jt, T, N - 1, np.array([T]), 1)
    dT[idx] = v[0]
    idx, v = _span_values(jt, T, N - 1, np.array([T]), 0)
    eT[idx] = v[0]
    A += np.outer(d0, d0)
    return dict(A=A, B=B, Me=Me, Ke=Ke, g=g, d0=d0, dT=dT, eT=eT)


def load_weights(jt, J, T):
    """W[i,n] = int lambda_n psi_i' e^{-t/T} dt, lambda_n the P1 hats of level J.

    Shape (2^jt + 1, 2^J + 1).  Integration over the finest elements."""
    Nf = 2 ** J
    hf = T / Nf
    ratio = 2 ** (J - jt)
    W = np.zeros((2 ** jt + 1, Nf + 1))
    for e in range(Nf):
        tq, wq = _elem_points(e * hf, (e + 1) * hf)
        w = wq * np.exp(-tq / T)
        lam_left = ((e + 1) * hf - tq) / hf
        lam_right = (tq - e * hf) / hf
        idx, v1 = _span_values(jt, T, e // ratio, tq, 1)
        for a, i in enumerate(idx):
            W[i, e] += np.sum(w * lam_left * v1[:, a])
            W[i, e + 1] += np.sum(w * lam_right * v1[:, a])
    return W


def eval_at_nodes(jt, J, T):
    """Psi[n,i] = psi_i(t_n) at the finest time nodes t_n = n T/2^J."""
    Nf = 2 ** J
    ratio = 2 ** (J - jt)
    Psi = np.zeros((Nf + 1, 2 ** jt + 1))
    for n in range(Nf + 1):
        e = min(n // ratio, 2 ** jt - 1)
        idx, v = _span_values(jt, T, e, np.array([n * T / Nf]), 0)
        Psi[n, idx] = v[0]
    return Psi


def eval_at(jt, T, t):
    """psi_i(t) at arbitrary points t in [0,T], shape (len(t), 2^jt + 1)."""
    return basis.time_basis(jt, T, t, 0)
