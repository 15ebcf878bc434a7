"""Combination index set of the sparse-grid method (oracle; test infrastructure).

Paper, Sec. 3.1, eq. (19) and Fig. 1: with finest level J the combination
formula sums the Galerkin solutions on V_{jx} (x) V_{J-jx} with coefficient +1
(jx = 0..J) and on V_{jx-1} (x) V_{J-jx} with coefficient -1 (jx = 1..J):
2J+1 solves on the diagonals jx+jt = J (+1) and jx+jt = J-1 (-1).

Level reading used by this library: the paper's level 0 has mesh size h_0 and
every experiment of Sec. 6 takes h_0 = 1/2 on the unit interval.  We index a
level by its number of uniform intervals, 2^j, so the paper's level j is our
level j+1.  With sparse level L the components are

    C_L = {(jx, jt) : jx >= 1, jt >= 1, jx + jt in {L, L-1}}

with sign +1 on jx+jt = L and -1 on jx+jt = L-1; this is eq. (19) with
J = L-2.  The finest level in space and in time is L-1.

Coarsest level (the h_0 of the coarse-mesh study of Sec. 6.3, Fig. 10):
h_0 = 2^-b0 makes the paper's level j our level j + b0.  Eq. (19) with its
levels shifted by b0 and the finest level kept at L-1 (J = L-1-b0) is

    C_{L,b0} = {(jx, jt) : jx >= b0, jt >= b0, jx + jt in {L-1+b0, L-2+b0}}

with the same signs; b0 = 1 is C_L above and b0 = L-1 the single full-grid
component (L-1, L-1).
"""


def components(L, b0=1):
    """List of (jx, jt, sign) for sparse level L >= 2 and coarsest level
    1 <= b0 <= L-1, eq. (19)."""
    if L < 2:
        raise ValueError("sparse level L must be >= 2")
    if not 1 <= b0 <= L - 1:
        raise ValueError("coarsest level b0 must be in [1, L-1]")
    out = []
    top = L - 1 + b0                      # jx + jt on the +1 diagonal
    for jx in range(b0, L):
        jt = top - jx
        if jt >= b0:
            out.append((jx, jt, +1))
    for jx in range(b0, L - 1):
        jt = top - 1 - jx
        if jt >= b0:
            out.append((jx, jt, -1))
    return out


def finest_level(L):
    """Finest level (space and time) touched by the components of C_L."""
    return L - 1


def n_space(jx, d):
    """Number of interior nodes of the P1 (d=1) / Q1 (d=2) space at level jx."""
    return (2 ** jx - 1) ** d


def n_time(jt):
    """Dimension of the quadratic C^1 spline space with w(0)=0: 2^jt + 1."""
    return 2 ** jt + 1


def n_sparse(L, d, b0=1):
    """Sum of component dimensions (the paper's N^sparse_DoFs, Sec. 3.2)."""
    return sum(n_space(jx, d) * n_time(jt) for jx, jt, _ in components(L, b0))


def n_full(L, d):
    """Number of nodal values of the finest full grid, including t = 0."""
    J = finest_level(L)
    return (2 ** J - 1) ** d * (2 ** J + 1)
