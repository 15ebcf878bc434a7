"""Write sampled oracle values of the 1-D differentiation workload.

Workload (``workloads.c4``): d=1, L=14, T=1, c piecewise constant on 8 cells
drawn from U[0.5, 2] (seed 0); observations U_obs = F(f_true, 0, 0) + noise
(sigma 1e-3); loss J = 1/2 sum (F(f, u0, v0) - U_obs)^2 over the finest-grid
nodes; gradient (dJ/df, dJ/du0) = F^T (U - U_obs) at f = a second Gaussian,
u0 = 0.1 sin(pi x), v0 = 0.

Everything is computed by the oracle (eq. 9 component solves, eq. 19
combination + lift, and the transposed map).  Seeded sample positions are
stored with their values.

Usage:  python tests/golden/make_c4_golden.py   (a few minutes)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import Problem  # noqa: E402

OUT = os.path.join(HERE, "c4_L14_samples.json")
NSAMP = 64


def main():
    t0 = time.perf_counter()
    spec, data = workloads.c4()
    prob = Problem(*spec.args())
    nt, ns = spec.nt(), spec.nx()
    zero = np.zeros(ns)
    U_obs = prob.forward(data["f_true"], zero, zero) + data["noise"].reshape(nt, ns)
    U = prob.forward(data["f"], data["u0"], data["v0"])
    r = U - U_obs
    J = 0.5 * float(np.sum(r * r))
    df, du0, dv0 = prob.adjoint(r)
    # componentwise magnitude of the expression du0 = sum_n r - sum_c
    # K_c^T (g^T z_c) (the adjoint of the lift and of the u0 load term):
    # |sum_n r| + sum_c |K_c|^T (|g|^T |z_c|), the scale of its rounding error
    du0_mag = np.abs(r.sum(axis=0))
    for jx, jt, s in prob.comps:
        y = s * (prob.psi_nodes(jt).T @ np.asarray((prob.phi(jx).T @ r.T).T))
        z = prob.solve(jx, jt, y, transpose=True)
        du0_mag += abs(prob.cross_stiff(jx)).T @ (np.abs(prob.tmat(jt)["g"]) @ np.abs(z))
    print(f"oracle done in {time.perf_counter() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(4321)
    pn = rng.integers(0, nt, NSAMP)
    pm = rng.integers(0, ns, NSAMP)
    ps = rng.integers(0, ns, NSAMP)
    out = dict(
        source="oracle/ forward (eq. 9, eq. 19 + lift) and adjoint; workloads.c4(L=14); "
               "written by tests/golden/make_c4_golden.py",
        loss=J, pos_n=pn.tolist(), pos_m=pm.tolist(), pos_s=ps.tolist(),
        U=U[pn, pm].tolist(), U_obs=U_obs[pn, pm].tolist(),
        df=df[pn, pm].tolist(), du0=du0[ps].tolist(), dv0=dv0[ps].tolist(),
        du0_mag=du0_mag[ps].tolist(),
        U_norm=float(np.linalg.norm(U)), df_norm=float(np.linalg.norm(df)),
        du0_norm=float(np.linalg.norm(du0)), dv0_norm=float(np.linalg.norm(dv0)))
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
