"""Pins of the oracle's L^2(Q_T) quadrature (Sec. 6.3 reports relative
L^2(Q_T) errors of the combined solution).

The rule (Gauss, nq_t points per finest time interval, nq_x per finest
element and space axis) is checked where its value is known in closed form:
a trilinear u (u^2 of degree 2 per variable, integrated exactly) against a
zero solution, a single space-time basis function (one uniform quadratic
B-spline, int B^2 = 11 tau / 20, times one hat, int phi^2 = 2 h / 3 per axis)
and the lift of a single nodal u0 value; with five points it equals the
rate-pinned l2_error of the same data.  The domain is not square and T != 1,
so a swapped axis or length changes the values."""

import numpy as np
import pytest

import workloads
from oracle import Problem, method

T = 0.7


def _zero_sols(orc):
    return [np.zeros((2 ** jt + 1, (2 ** jx - 1) ** orc.d)) for (jx, jt, s) in orc.comps]


@pytest.mark.parametrize("d", [1, 2])
def test_rule_exact_for_trilinear(d):
    lengths = [1.0, 0.8][:d]
    spec = workloads.Spec(d, lengths, [1] * d, [1.0], T, 4)
    orc = Problem(*spec.args())
    u = (lambda t, x: t * x) if d == 1 else (lambda t, x, y: t * x * y)
    e, n = method.l2_error_rule(orc, _zero_sols(orc), np.zeros(spec.space_shape()), u)
    want = T ** 3 / 3 * np.prod([a ** 3 / 3 for a in lengths])
    assert abs(n - want) <= 1e-14 * want and abs(e - want) <= 1e-14 * want


@pytest.mark.parametrize("d", [1, 2])
def test_rule_single_basis_function(d):
    """u_h = psi_q (x) phi_K (one component, one coefficient), u = 0: the
    integral of its square is (11 tau / 20) prod (2 h_a / 3)."""
    lengths = [1.0, 0.8][:d]
    spec = workloads.Spec(d, lengths, [1] * d, [1.0], T, 6)
    orc = Problem(*spec.args())
    sols = _zero_sols(orc)
    c = next(i for i, (jx, jt, s) in enumerate(orc.comps) if jt >= 3 and jx >= 2)
    jx, jt, _ = orc.comps[c]
    n = 2 ** jx - 1
    K = n // 2 if d == 1 else (n // 2) * n + n // 3   # an interior hat (row n//2, column n//3)
    sols[c][3, K] = 1.0                                 # B-spline of index 3: interior
    zero = (lambda t, x: 0.0 * t * x) if d == 1 else (lambda t, x, y: 0.0 * t * x * y)
    e, nrm = method.l2_error_rule(orc, sols, np.zeros(spec.space_shape()), zero)
    want = 11.0 / 20.0 * T / 2 ** jt * np.prod([2.0 / 3.0 * a / 2 ** jx for a in lengths])
    assert nrm == 0.0
    assert abs(e - want) <= 1e-13 * want


def test_rule_lift_of_one_nodal_value():
    """No component contribution, u0 = one finest nodal value 1, u = 0: the
    lift is that finest hat for all t, so the integral is T (2 hx / 3)(2 hy / 3)."""
    spec = workloads.Spec(2, [1.0, 0.8], [1, 1], [1.0], T, 5)
    orc = Problem(*spec.args())
    u0 = np.zeros(spec.space_shape())
    u0[7, 4] = 1.0
    e, _ = method.l2_error_rule(orc, _zero_sols(orc), u0, lambda t, x, y: 0.0 * t * x * y)
    h = [a / 2 ** orc.J for a in (1.0, 0.8)]
    want = T * (2.0 * h[0] / 3.0) * (2.0 * h[1] / 3.0)
    assert abs(e - want) <= 1e-13 * want


@pytest.mark.parametrize("d", [1, 2])
def test_rule_with_five_points_is_the_rate_pinned_error(d):
    spec = workloads.Spec(d, [1.0, 0.8][:d], [1] * d, [1.0], T, 5)
    data = workloads.random_data(spec, 11)
    orc = Problem(*spec.args())
    sols = orc.component_solutions(data["f"], np.zeros(spec.space_shape()), data["v0"])
    u = (lambda t, x: np.sin(2 * x + t)) if d == 1 else \
        (lambda t, x, y: np.sin(2 * x + t) * np.cos(3 * y))
    e1, n1 = method.l2_error(orc, sols, u)
    e2, n2 = method.l2_error_rule(orc, sols, np.zeros(spec.space_shape()), u, 5, 5)
    assert abs(e2 - e1 ** 2) <= 1e-13 * e1 ** 2 and abs(n2 - n1 ** 2) <= 1e-13 * n1 ** 2


def test_rule_lift_against_a_linear_function_of_x():
    """u = x, u_h = the finest hat of node (row 7, column 4) for all t:
    int (x - phi)^2 = T (Lx^3 Ly / 3 - 2 x_K hx hy + (2 hx / 3)(2 hy / 3)),
    x_K = 5 hx (interior node 4 is the fifth).  Exact for the rule (both
    factors are linear on every finest cell); an x/y mix-up of the nodal
    array or the points moves x_K or the domain lengths."""
    spec = workloads.Spec(2, [1.0, 0.8], [1, 1], [1.0], T, 5)
    orc = Problem(*spec.args())
    u0 = np.zeros(spec.space_shape())
    u0[7, 4] = 1.0
    e, n = method.l2_error_rule(orc, _zero_sols(orc), u0, lambda t, x, y: x + 0.0 * t * y)
    hx, hy = 1.0 / 2 ** orc.J, 0.8 / 2 ** orc.J
    want = T * (0.8 / 3.0 - 2.0 * 5 * hx * hx * hy + (2 * hx / 3) * (2 * hy / 3))
    assert abs(n - T * 0.8 / 3.0) <= 1e-14 and abs(e - want) <= 1e-13 * want
