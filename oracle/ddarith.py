"""Double-double arithmetic on numpy arrays (oracle; test infrastructure).

Error-free transformations (Knuth's two-sum, Dekker's splitting product)
vectorised over arrays; a value is a pair (hi, lo) with |lo| <= ulp(hi)/2.
Used for the residual of the iterative refinement, which must be formed with
the exact (double-double) time matrices.
"""

import numpy as np

_SPLITTER = 134217729.0  # 2^27 + 1


def split(a):
    c = _SPLITTER * a
    hi = c - (c - a)
    return hi, a - hi


def two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def two_prod(a, b):
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


def add(xh, xl, yh, yl):
    s, e = two_sum(xh, yh)
    e = e + (xl + yl)
    return two_sum(s, e)


def mul(xh, xl, yh, yl):
    """(xh + xl)(yh + yl) to double-double accuracy."""
    p, e = two_prod(xh, yh)
    e = e + (xh * yl + xl * yh)
    return two_sum(p, e)


def zeros(shape):
    return np.zeros(shape), np.zeros(shape)
