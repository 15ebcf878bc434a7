"""Pins of the oracle's coarsest-level parameter b0 (h_0 = 2^-b0, the
coarse-mesh study of Sec. 6.3, Fig. 10).

* The index set and signs are eq. (19) written in the paper's own levels
  (0..J, +1 on V_j (x) V_{J-j} for j = 0..J, -1 on V_{j-1} (x) V_{J-j} for
  j = 1..J) and moved to this library's levels by the shift h_0 = 2^-b0
  (paper level j = level j + b0), with the finest level J + b0 = L - 1.
* b0 = L-1 leaves one component, the finest full grid: the combined
  solution equals full_grid(L-1) (eq. 10), on a variable-speed case.
* A manufactured smooth solution: the relative L^2(Q_T) error of the
  combination with b0 = 2 falls at the sparse-grid rate when L grows (the
  finest mesh halves), so a wrong component or sign (which leaves an O(1)
  term) fails it.
"""

import numpy as np
import pytest

import workloads
from oracle import Problem, levels, method


def _paper_set(J, b0):
    out = set()
    for j in range(0, J + 1):
        out.add((j + b0, J - j + b0, +1))
    for j in range(1, J + 1):
        out.add((j - 1 + b0, J - j + b0, -1))
    return out


@pytest.mark.parametrize("b0", [1, 2, 3])
@pytest.mark.parametrize("J", [0, 1, 2, 4])
def test_index_set_is_eq19_in_shifted_levels(J, b0):
    L = J + b0 + 1
    comps = levels.components(L, b0)
    assert len(comps) == 2 * J + 1 == len(set(comps))
    assert set(comps) == _paper_set(J, b0)
    assert max(max(a, b) for a, b, _ in comps) == L - 1
    assert min(min(a, b) for a, b, _ in comps) == b0


def test_default_is_b0_one():
    for L in range(2, 9):
        assert levels.components(L) == levels.components(L, 1)
    assert levels.n_sparse(10, 2) == levels.n_sparse(10, 2, 1)


def test_invalid_offsets_are_refused():
    with pytest.raises(ValueError):
        levels.components(5, 0)
    with pytest.raises(ValueError):
        levels.components(5, 5)


@pytest.mark.parametrize("d", [1, 2])
def test_single_component_is_the_full_grid(d):
    L = 4
    lengths = [1.0, 0.8][:d]
    ncell = [2] * d
    cv = [1.0, 0.6, 1.4, 0.8][:2 ** d]
    spec = workloads.Spec(d, lengths, ncell, cv, 0.9, L)
    data = workloads.random_data(spec, 5)
    orc = Problem(*spec.args(), b0=L - 1)
    assert orc.comps == [(L - 1, L - 1, +1)]
    U = orc.forward(data["f"], data["u0"], data["v0"]).reshape(spec.shape())
    ref = orc.full_grid(L - 1, data["f"], data["u0"], data["v0"]).reshape(spec.shape())
    assert np.max(np.abs(U - ref)) <= 1e-13 * np.max(np.abs(ref))


def _manufactured_error(L, b0):
    """Relative L^2(Q_T) error of the combination for the 1-D solution
    u = sin(pi x) sin^2(t) (u(0) = u_t(0) = 0) with its exact load."""
    spec = workloads.Spec(1, [1.0], [1], [1.0], 1.0, L)
    orc = Problem(*spec.args(), b0=b0)
    u = lambda t, x: np.sin(np.pi * x) * np.sin(t) ** 2
    f = lambda t, x: np.sin(np.pi * x) * (2 * np.cos(2 * t) + np.pi ** 2 * np.sin(t) ** 2)
    zero = lambda x: 0.0 * x
    sols = []
    for jx, jt, _ in orc.comps:
        b = method.load_exact(orc, jx, jt, f, zero, zero, lambda x: [0.0 * x])
        sols.append(orc.solve(jx, jt, b))
    e, n = method.l2_error(orc, sols, u)
    return e / n


def test_offset_combination_converges():
    e = [_manufactured_error(L, 2) for L in (6, 7, 8)]
    assert e[0] < 2e-3
    # the finest mesh halves per step: second order up to the sparse-grid log factor
    assert e[1] / e[0] < 0.4 and e[2] / e[1] < 0.4
