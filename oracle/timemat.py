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

Local coordinates.  Basis functions are always evaluated on one element at
its local coordinate s in [0,1], with the knots measured in units of h from
the element start (small integers).  Evaluating at absolute times instead
would subtract nearly equal numbers t - tau and lose about log10(N) digits.

Exact time matrices.  The discrete solution on long time levels is very
sensitive to last-bit perturbations of the entries of A and B (the system
matrix is nearly singular in its own basis), so ``time_matrices_dd``
computes them with 40-digit mpmath arithmetic and returns each as a pair of
doubles (hi, lo) with hi + lo correct to about 32 digits.  On element e,
t = T (e + s)/N, so e^{-t/T} = e^{-e/N} e^{-s/N}; the element integral is
e^{-e/N} times an integral over s that depends only on the element's knot
pattern, which repeats for all interior elements.

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


def _ref_knots_shifted(jt, e):
    """Clamped knots of level jt in units of h, shifted by -e (element e)."""
    N = 2 ** jt
    return np.array([0, 0, 0] + list(range(1, N)) + [N, N, N], dtype=np.float64) - e


def _span_values(jt, T, e, s, deriv):
    """psi_i^{(deriv)} on element e of level jt at local coordinates s in [0,1].

    Element e = [e h, (e+1) h] is knot span e + 2; the nonzero B-splines there
    are B_e, B_{e+1}, B_{e+2}, i.e. psi_{e-1}, psi_e, psi_{e+1} (psi_{-1} = B_0
    is the dropped function).  Returns (indices, values)."""
    h = T / 2 ** jt
    vals = basis.local_basis(_ref_knots_shifted(jt, e), 2, e + 2, s, deriv)
    vals = vals / h ** deriv
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
    sq, wq = _elem_points(0.0, 1.0)
    for e in range(N):
        w = h * wq * np.exp(-(e + sq) / N)
        idx, v0 = _span_values(jt, T, e, sq, 0)
        _, v1 = _span_values(jt, T, e, sq, 1)
        _, v2 = _span_values(jt, T, e, sq, 2)
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
    idx, v = _span_values(jt, T, N - 1, np.array([1.0]), 1)
    dT[idx] = v[0]
    idx, v = _span_values(jt, T, N - 1, np.array([1.0]), 0)
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
    sq, wq = _elem_points(0.0, 1.0)
    lam_left = 1.0 - sq
    lam_right = sq
    for e in range(Nf):
        w = hf * wq * np.exp(-(e + sq) / Nf)
        ec = e // ratio
        sc = ((e - ec * ratio) + sq) / ratio   # local coordinate on the coarse element
        idx, v1 = _span_values(jt, T, ec, sc, 1)
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
        idx, v = _span_values(jt, T, e, np.array([(n - e * ratio) / ratio]), 0)
        Psi[n, idx] = v[0]
    return Psi


_DD_CACHE = {}


def _mp_local(knots, s, mp):
    """B_{span-2..span} and their first two derivatives (knot units) at s,
    Cox-de Boor in mpmath; knots are the 6 knots around the span, shifted."""
    # span index 2 in this 6-knot window (knots[2] <= s < knots[3])
    vals = {2: mp.mpf(1)}
    out = []
    for deriv in range(3):
        v = {2: mp.mpf(1)}
        for k in range(1, 3):
            derivative = k > 2 - deriv
            new = {}
            for i in range(2 - k, 3):
                lo = v.get(i, mp.mpf(0))
                hi = v.get(i + 1, mp.mpf(0))
                d1 = knots[i + k] - knots[i]
                d2 = knots[i + k + 1] - knots[i + 1]
                if derivative:
                    a = mp.mpf(k) / d1 if d1 > 0 else 0
                    b = mp.mpf(k) / d2 if d2 > 0 else 0
                    new[i] = a * lo - b * hi
                else:
                    a = (s - knots[i]) / d1 if d1 > 0 else 0
                    b = (knots[i + k + 1] - s) / d2 if d2 > 0 else 0
                    new[i] = a * lo + b * hi
            v = new
        out.append([v[i] for i in range(0, 3)])
    del vals
    return out


def band_to_dense(band):
    """(n,5) band with entry (i, i+k-2) at [i, k] -> dense (n,n)."""
    n = band.shape[0]
    D = np.zeros((n, n))
    for k in range(5):
        off = k - 2
        i = np.arange(max(0, -off), min(n, n - off))
        D[i, i + off] = band[i, k]
    return D


def time_vectors(jt, T):
    """g[i] = int psi_i' e^{-t/T} dt and d0[i] = psi_i'(0) (O(2^jt) work)."""
    N = 2 ** jt
    h = T / N
    g = np.zeros(N + 1)
    sq, wq = _elem_points(0.0, 1.0)
    for e in range(N):
        w = h * wq * np.exp(-(e + sq) / N)
        idx, v1 = _span_values(jt, T, e, sq, 1)
        for a, i in enumerate(idx):
            g[i] += np.sum(w * v1[:, a])
    d0 = np.zeros(N + 1)
    idx, v = _span_values(jt, T, 0, np.array([0.0]), 1)
    d0[idx] = v[0]
    return g, d0


def _bget(M, i, j):
    k = j - i + 2
    return M[i][k] if 0 <= k < 5 else 0


def _max_identity_defect(n, lhs, rhs, mp):
    """max |lhs - rhs| / max |rhs| over the band (|i-j| <= 2)."""
    worst, scale = mp.mpf(0), mp.mpf(0)
    for i in range(n):
        for j in range(max(0, i - 2), min(n, i + 3)):
            r = rhs(i, j)
            worst = max(worst, abs(lhs(i, j) - r))
            scale = max(scale, abs(r))
    return float(worst / scale)


def time_matrices_dd(jt, T):
    """A and B of eq. (30) to ~32 digits, banded: dict with A_hi, A_lo, B_hi,
    B_lo of shape (2^jt+1, 5), entry (i, i+k-2) at [i, k]."""
    key = (jt, float(T))
    if key in _DD_CACHE:
        return _DD_CACHE[key]
    import mpmath
    mp = mpmath.mp.clone() if hasattr(mpmath.mp, "clone") else mpmath.mp
    old = mp.dps
    mp.dps = 40
    try:
        N = 2 ** jt
        n = N + 1
        gl = mpmath.calculus.quadrature.GaussLegendre(mp)
        nodes = [((x + 1) / 2, w / 2) for x, w in gl.calc_nodes(3, mp.prec)]  # 12 points
        lam = mp.mpf(1) / N
        local_cache = {}
        A = [[mp.mpf(0)] * 5 for _ in range(n)]
        B = [[mp.mpf(0)] * 5 for _ in range(n)]
        Me = [[mp.mpf(0)] * 5 for _ in range(n)]   # (psi_j, psi_i)_e in units of h
        Ke = [[mp.mpf(0)] * 5 for _ in range(n)]   # (psi_j', psi_i')_e in units of 1/h
        E1 = mp.exp(-lam)
        Ee = mp.mpf(1)
        full = [0, 0, 0] + list(range(1, N)) + [N, N, N]
        for e in range(N):
            window = tuple(k - e for k in full[e:e + 6])  # knots tau_e..tau_{e+5}
            if window not in local_cache:
                a_loc = [[mp.mpf(0)] * 3 for _ in range(3)]
                b_loc = [[mp.mpf(0)] * 3 for _ in range(3)]
                m_loc = [[mp.mpf(0)] * 3 for _ in range(3)]
                k_loc = [[mp.mpf(0)] * 3 for _ in range(3)]
                for s, w in nodes:
                    v, d1, d2 = _mp_local([mp.mpf(k) for k in window], s, mp)
                    wt = w * mp.exp(-lam * s)
                    for fi in range(3):
                        for fj in range(3):
                            a_loc[fi][fj] += wt * d2[fj] * d1[fi]
                            b_loc[fi][fj] += wt * v[fj] * d1[fi]
                            m_loc[fi][fj] += wt * v[fj] * v[fi]
                            k_loc[fi][fj] += wt * d1[fj] * d1[fi]
                local_cache[window] = (a_loc, b_loc, m_loc, k_loc)
            a_loc, b_loc, m_loc, k_loc = local_cache[window]
            for fi in range(3):
                i = e + fi - 1
                if i < 0:
                    continue
                for fj in range(3):
                    j = e + fj - 1
                    if j < 0:
                        continue
                    A[i][j - i + 2] += Ee * a_loc[fi][fj]
                    B[i][j - i + 2] += Ee * b_loc[fi][fj]
                    Me[i][j - i + 2] += Ee * m_loc[fi][fj]
                    Ke[i][j - i + 2] += Ee * k_loc[fi][fj]
            Ee = Ee * E1
        A[0][2] += 4  # psi_0'(0)^2 in knot units (slope 2/h)
        # B_N(T) = 1, slopes at T: psi_N' = 2/h, psi_{N-1}' = -2/h (knot units)
        eT = [mp.mpf(0)] * n
        eT[N] = mp.mpf(1)
        dT = [mp.mpf(0)] * n
        dT[N], dT[N - 1] = mp.mpf(2), mp.mpf(-2)
        Tm = mp.mpf(float(T))
        scale = (mp.mpf(N) / Tm) ** 2
        out = {"identity_B": _max_identity_defect(
                   n, lambda i, j: _bget(B, i, j) + _bget(B, j, i),
                   lambda i, j: _bget(Me, i, j) * Tm / N / Tm + eT[i] * eT[j] / mp.e, mp),
               "identity_A": _max_identity_defect(
                   n, lambda i, j: (_bget(A, i, j) + _bget(A, j, i)) * scale,
                   lambda i, j: (_bget(Ke, i, j) * N / Tm / Tm
                                 + (dT[i] * dT[j] / mp.e + (4 if i == j == 0 else 0))
                                 * scale), mp)}
        for name, M, sc in (("A", A, scale), ("B", B, mp.mpf(1))):
            hi = np.zeros((n, 5))
            lo = np.zeros((n, 5))
            for i in range(n):
                for k in range(5):
                    if 0 <= i + k - 2 < n:
                        x = M[i][k] * sc
                        h_ = float(x)
                        hi[i, k] = h_
                        lo[i, k] = float(x - h_)
            out[name + "_hi"] = hi
            out[name + "_lo"] = lo
    finally:
        mp.dps = old
    _DD_CACHE[key] = out
    return out


def eval_at(jt, T, t):
    """psi_i(t) at arbitrary points t in [0,T], shape (len(t), 2^jt + 1)."""
    return basis.time_basis(jt, T, t, 0)
