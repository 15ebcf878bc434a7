"""1-D configurations with a piecewise-constant wave speed, on the GPU.

* two-speed medium (c = 1 on (0, 1/2), 1/2 on (1/2, 1); L = 12, T = 2): forward
  and adjoint element by element against the oracle; the distance to the
  full-grid solution at level 8/8 is reported (a discretisation error, not a
  parity check);
* differentiation workload (8 random speeds, L = 14): gradient of the
  least-squares misfit through torch.autograd (hand-written adjoint) against
  the oracle's gradient (stored samples, written by
  tests/golden/make_c4_golden.py; du0 within a few units of rounding of its
  componentwise magnitude, see the test) and against central finite
  differences on 32 unit directions (h = 1e-6 as in the workload's
  definition, bounded by the rounding floor of the loss, and h = 1e-2, where
  the exact quadratic makes a tight check possible).
"""

import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import Problem

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN_C4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "c4_L14_samples.json")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).reshape(-1), np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_two_speed_medium_parity():
    torch = _torch()
    import paper_2606_09688_amd as sg
    spec, data = workloads.c2()
    g = workloads.random_data(spec, 12)["g"]
    print("two-speed medium: d=1 L=12 T=2", flush=True)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    sv = sg.SparseGridWave(*spec.args())
    U = sv.solve(dev(data["f"]), dev(data["u0"]), dev(data["v0"])).cpu().numpy()
    df, du0, dv0 = (x.cpu().numpy() for x in sv.adjoint(dev(g)))
    orc = Problem(*spec.args())
    U_ref = orc.forward(data["f"], data["u0"], data["v0"]).reshape(spec.shape())
    eU = _rel(U, U_ref)
    print(f"  forward rel l2 {eU:.3e}", flush=True)
    assert eU <= TOL
    df_ref, du0_ref, dv0_ref = orc.adjoint(g)
    for name, got, ref in (("df", df, df_ref), ("du0", du0, du0_ref), ("dv0", dv0, dv0_ref)):
        e = _rel(got, ref)
        print(f"  adjoint {name} rel l2 {e:.3e}", flush=True)
        assert e <= TOL, name
    # reported: sparse-grid solution vs the full grid P_{8,8} at its nodes
    P88 = orc.full_grid(8, data["f"], data["u0"], data["v0"]).reshape(spec.shape())
    step = 2 ** (spec.J - 8)
    sub = (slice(None, None, step), slice(step - 1, None, step))
    print(f"  |U - P_88| / |P_88| on the level-8 nodes: {_rel(U[sub], P88[sub]):.3e}", flush=True)


def test_gradient_of_misfit():
    torch = _torch()
    import paper_2606_09688_amd as sg
    with open(GOLDEN_C4) as fh:
        gold = json.load(fh)
    spec, data = workloads.c4()
    print("differentiation workload: d=1 L=14, 8 speeds", flush=True)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    sv = sg.SparseGridWave(*spec.args())
    zero = torch.zeros(spec.space_shape(), dtype=torch.float64, device="cuda")
    U_obs = sv.solve(dev(data["f_true"]), zero, zero) + dev(data["noise"])
    f = dev(data["f"]).requires_grad_(True)
    u0 = dev(data["u0"]).requires_grad_(True)
    v0 = dev(data["v0"])

    def loss(f_, u0_):
        U = sg.sgwave(sv, f_, u0_, v0)
        return 0.5 * torch.sum((U - U_obs) ** 2)

    J = loss(f, u0)
    J.backward()
    gf, gu0 = f.grad.detach(), u0.grad.detach()
    # against the oracle (stored samples of its gradient)
    pn, pm, ps = (np.asarray(gold[k]) for k in ("pos_n", "pos_m", "pos_s"))
    edf = _rel(gf.cpu().numpy()[pn, pm], gold["df"])
    gu = gu0.cpu().numpy()[ps]
    edu = _rel(gu, gold["du0"])
    # du0 = sum_n r - sum_c K_c^T (g^T z_c) (adjoint of the lift and of the u0
    # load term).  At this workload the finest-level summand applies K to a
    # field ~1e7 larger than the result, and the summands cancel further, so
    # the FP64 rounding of the expression itself (on either side) is ~1e-9 of
    # |du0|: du0 is held to a few units of rounding of its componentwise
    # magnitude |sum_n r| + sum_c |K_c|^T (|g|^T |z_c|) (stored by the oracle;
    # ~8.5e7 |du0| at the sampled nodes), i.e. to ~7e-7 relative, instead.
    eps = 2.0 ** -52
    edu_ulp = float(np.linalg.norm(gu - np.asarray(gold["du0"])) /
                    (eps * np.linalg.norm(gold["du0_mag"])))
    eJ = abs(float(J.detach()) - gold["loss"]) / abs(gold["loss"])
    print(f"  vs oracle: loss {eJ:.2e}  df {edf:.2e}  du0 {edu:.2e} "
          f"({edu_ulp:.2f} eps of its componentwise magnitude)", flush=True)
    assert edf <= TOL and eJ <= TOL
    assert edu <= TOL or edu_ulp <= 8.0
    # central finite differences on unit directions over (f, u0).  J is
    # quadratic, so the difference quotient has no truncation error at any h;
    # its error is the rounding of the two loss values, ~eps |J| / h.  At
    # h = 1e-6 the check is bounded by that floor; at h = 1e-2 the floor is
    # far below 1e-6 of the directional derivative and the check is tight.
    Jv = abs(float(J.detach()))
    with torch.no_grad():
        for h, tight in ((1e-6, False), (1e-2, True)):
            worst = 0.0
            for k in range(32):
                d_f, d_u0 = workloads.c4_direction(spec, k)
                d_f, d_u0 = dev(d_f), dev(d_u0)
                jp = float(loss(f + h * d_f, u0 + h * d_u0))
                jm = float(loss(f - h * d_f, u0 - h * d_u0))
                fd = (jp - jm) / (2 * h)
                an = float(torch.sum(gf * d_f) + torch.sum(gu0 * d_u0))
                floor = 1e3 * eps * Jv / h
                assert abs(fd - an) <= 1e-6 * abs(an) + (0.0 if tight else floor), (h, k, fd, an)
                worst = max(worst, abs(fd - an) / max(abs(an), 1e-300))
            print(f"  finite differences (32 directions, h = {h:g}): worst rel {worst:.2e} "
                  f"(|J| = {Jv:.3e})", flush=True)


def test_adjoint_of_a_stored_cotangent_at_full_size():
    """The differentiation workload's adjoint on the SAME seeded cotangent as
    the oracle (workloads.c4_cotangent; make_sketch_golden.py c4), so that no
    forward rounding enters the comparison: du0 and dv0 element by element
    in full, df and the forward U at the gradient point through whole-array
    sketches, all to 1e-10 relative l2."""
    torch = _torch()
    import paper_2606_09688_amd as sg
    from sketchcheck import sketch_error
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_sketch.json")
    with open(path) as fh:
        gold = json.load(fh)
    spec, data = workloads.c4()
    print("differentiation workload: adjoint of a stored cotangent, d=1 L=14", flush=True)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    sv = sg.SparseGridWave(*spec.args())
    U = sv.solve(dev(data["f"]), dev(data["u0"]), dev(data["v0"]))
    df, du0, dv0 = sv.adjoint(dev(workloads.c4_cotangent(spec)))
    torch.cuda.synchronize()
    edu = _rel(du0.cpu().numpy(), np.asarray(gold["du0_full"]))
    edv = _rel(dv0.cpu().numpy(), np.asarray(gold["dv0_full"]))
    eU, _ = sketch_error(U, gold["U"])
    edf, _ = sketch_error(df, gold["df"])
    print(f"  U {eU:.2e}  df {edf:.2e}  du0 {edu:.2e}  dv0 {edv:.2e}", flush=True)
    assert max(eU, edf, edu, edv) <= TOL
