"""Basis functions (oracle; test infrastructure).

Time (paper Sec. 2.2: V^t_{jt} subset of H^2_{0,.}(0,T); Rem. 1 / Table 1:
C^1 splines of even degree satisfy assumption (14); Sec. 3.2 dimension
formula with p_t = 2, r_t = 1): quadratic B-splines on the uniform clamped
knot vector of 2^jt intervals of (0,T),

    tau = (0, 0, 0, h, 2h, ..., (N-1)h, T, T, T),   N = 2^jt, h = T/N,

give N+2 functions B_0..B_{N+1}.  Only B_0 is nonzero at t = 0, so dropping
it imposes w(0) = 0 and leaves the basis psi_i = B_{i+1}, i = 0..N
(dimension N+1).  Evaluation is the Cox-de Boor recursion with its standard
derivative formula.

Space (Sec. 2.2: V^x_{jx} subset of H^1_0(Omega)): continuous piecewise
linear hats on 2^jx uniform intervals per axis, interior nodes only; in 2-D
the tensor-product (Q1) hats.
"""

import numpy as np


def clamped_knots(jt, T):
    """Knot vector of the clamped uniform quadratic spline space at level jt."""
    N = 2 ** jt
    h = T / N
    inner = [k * h for k in range(1, N)]
    return np.array([0.0, 0.0, 0.0] + inner + [T, T, T], dtype=np.float64)


def _bspline_all(knots, p, t, deriv):
    """Values (deriv=0,1,2) of all degree-p B-splines of `knots` at points t.

    Cox-de Boor: B_{i,0} is the indicator of [tau_i, tau_{i+1}) (the last
    non-empty interval is closed on the right so that t = T is covered);
    B_{i,k} = w1 B_{i,k-1} + w2 B_{i+1,k-1} with 0/0 := 0.  Derivatives use
    B'_{i,k} = k (B_{i,k-1}/(tau_{i+k}-tau_i) - B_{i+1,k-1}/(tau_{i+k+1}-tau_{i+1})).
    Returns an array of shape (len(t), len(knots)-p-1).
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    m = len(knots) - 1
    # degree-0 indicators
    B = np.zeros((len(t), m), dtype=np.float64)
    last = max(i for i in range(m) if knots[i] < knots[i + 1])
    for i in range(m):
        if knots[i] < knots[i + 1]:
            inside = (t >= knots[i]) & (t < knots[i + 1])
            if i == last:
                inside |= t == knots[i + 1]
            B[:, i] = inside.astype(np.float64)

    def raise_degree(B, k, derivative):
        n = B.shape[1] - 1
        out = np.zeros((len(t), n), dtype=np.float64)
        for i in range(n):
            d1 = knots[i + k] - knots[i]
            d2 = knots[i + k + 1] - knots[i + 1]
            if derivative:
                a = k / d1 if d1 > 0 else 0.0
                b = k / d2 if d2 > 0 else 0.0
                out[:, i] = a * B[:, i] - b * B[:, i + 1]
            else:
                a = (t - knots[i]) / d1 if d1 > 0 else 0.0
                b = (knots[i + k + 1] - t) / d2 if d2 > 0 else 0.0
                out[:, i] = a * B[:, i] + b * B[:, i + 1]
        return out

    # values up to degree p - deriv, then differentiate `deriv` times
    for k in range(1, p - deriv + 1):
        B = raise_degree(B, k, derivative=False)
    for k in range(p - deriv + 1, p + 1):
        B = raise_degree(B, k, derivative=True)
    return B


def local_basis(knots, p, s, t, deriv=0):
    """The p+1 B-splines B_{s-p}..B_s (deriv-th derivative) for t in span s.

    Same Cox-de Boor recursion as `_bspline_all`, evaluated only on the
    indices that are nonzero on the knot span [tau_s, tau_{s+1}) (t must lie
    in its closure).  Returns an array of shape (len(t), p+1).
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    vals = {s: np.ones_like(t)}
    for k in range(1, p + 1):
        derivative = k > p - deriv
        new = {}
        for i in range(s - k, s + 1):
            lo = vals.get(i, 0.0)
            hi = vals.get(i + 1, 0.0)
            d1 = knots[i + k] - knots[i]
            d2 = knots[i + k + 1] - knots[i + 1]
            if derivative:
                a = k / d1 if d1 > 0 else 0.0
                b = k / d2 if d2 > 0 else 0.0
                new[i] = a * lo - b * hi
            else:
                a = (t - knots[i]) / d1 if d1 > 0 else 0.0
                b = (knots[i + k + 1] - t) / d2 if d2 > 0 else 0.0
                new[i] = a * lo + b * hi
        vals = new
    return np.stack([vals[i] * np.ones_like(t) for i in range(s - p, s + 1)],
                    axis=1)


def time_basis(jt, T, t, deriv=0):
    """psi_i^{(deriv)}(t) for i = 0..2^jt (i.e. B_1..B_{N+1}), shape (len(t), N+1)."""
    knots = clamped_knots(jt, T)
    return _bspline_all(knots, 2, t, deriv)[:, 1:]


def time_basis_full(jt, T, t, deriv=0):
    """All N+2 clamped quadratic B-splines including the dropped B_0."""
    return _bspline_all(clamped_knots(jt, T), 2, t, deriv)


def hat_1d(j, length, x):
    """P1 hats of the interior nodes x_k = k*h (k = 1..2^j-1) at points x.

    Shape (len(x), 2^j - 1).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = 2 ** j
    h = length / n
    nodes = h * np.arange(1, n)
    return np.maximum(0.0, 1.0 - np.abs(x[:, None] - nodes[None, :]) / h)


def hat_1d_node(j, length, k, x):
    """Value of the single hat of interior node k (x_k = k h, 1 <= k < 2^j)."""
    x = np.asarray(x, dtype=np.float64)
    h = length / 2 ** j
    return np.maximum(0.0, 1.0 - np.abs(x - k * h) / h)


def hat_1d_node_deriv(j, length, k, x):
    """Derivative of the hat of interior node k at points x (not on a node)."""
    x = np.asarray(x, dtype=np.float64)
    h = length / 2 ** j
    dist = x - k * h
    return np.where(np.abs(dist) < h, -np.sign(dist) / h, 0.0)


def hat_1d_deriv(j, length, x):
    """Derivatives of the interior P1 hats at points x (no point on a node)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = 2 ** j
    h = length / n
    nodes = h * np.arange(1, n)
    dist = x[:, None] - nodes[None, :]
    inside = np.abs(dist) < h
    return np.where(inside, -np.sign(dist) / h, 0.0)


def p1_time_hat(J, T, t):
    """P1 hats lambda_n of the time nodes t_n = n T/2^J, n = 0..2^J (incl. ends)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = 2 ** J
    h = T / n
    nodes = h * np.arange(0, n + 1)
    return np.maximum(0.0, 1.0 - np.abs(t[:, None] - nodes[None, :]) / h)
