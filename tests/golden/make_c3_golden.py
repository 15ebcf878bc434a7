"""Write sampled oracle values of the full-size 2-D benchmark workload.

Workload: d=2, Omega=(0,1)^2, L=10, c=1, T=1, manufactured
u = sin(pi x) sin(pi y) sin(pi t) (f = pi^2 u, u0 = 0, v0 = pi sin sin) and the
adjoint cotangent g ~ N(0,1), seed 0 (``workloads.c3``).

Everything here comes from the oracle (``oracle/``): the component loads and
solutions of eq. (9), the combination of eq. (19) plus the lift, and the
adjoint of the whole forward map.  The full arrays are far too large for a
fixture, so seeded sample positions are stored with their values.

Usage:  python tests/golden/make_c3_golden.py   (several minutes, ~10 GB RAM)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import Problem  # noqa: E402

OUT = os.path.join(HERE, "c3_L10_samples.json")
NSAMP = 64      # fine-grid samples per output array
NCOMP = 8       # samples per component array


def main():
    t0 = time.perf_counter()
    spec, data = workloads.c3(L=10)
    prob = Problem(*spec.args())
    nt, ns = spec.nt(), spec.nx() ** spec.d
    f = data["f"].reshape(nt, ns)
    u0 = data["u0"].reshape(ns)
    v0 = data["v0"].reshape(ns)
    g = data["g"].reshape(nt, ns)
    rng = np.random.default_rng(12345)
    pos_n = rng.integers(0, nt, NSAMP)
    pos_m = rng.integers(0, ns, NSAMP)
    pos_s = rng.integers(0, ns, NSAMP)

    comps = []
    U_s = u0[pos_m].copy()
    for jx, jt, s in prob.comps:
        b = prob.load(jx, jt, f, u0, v0)
        u = prob.solve(jx, jt, b)
        cpos = rng.integers(0, u.size, NCOMP)
        comps.append(dict(jx=jx, jt=jt, sign=s, pos=cpos.tolist(),
                          load=b.reshape(-1)[cpos].tolist(), sol=u.reshape(-1)[cpos].tolist(),
                          load_norm=float(np.linalg.norm(b)), sol_norm=float(np.linalg.norm(u))))
        # U at the sample points: psi^jt_i(t_n) phi^jx_k(x_m) u[i, k]
        Psi = prob.psi_nodes(jt)
        Phi = prob.phi(jx).tocsr()
        for k in range(NSAMP):
            U_s[k] += s * float(Psi[pos_n[k]] @ (u @ Phi[pos_m[k]].toarray().reshape(-1)))
        print(f"component ({jx},{jt}) done, {time.perf_counter() - t0:.0f} s", flush=True)
    df, du0, dv0 = prob.adjoint(g)
    print(f"adjoint done, {time.perf_counter() - t0:.0f} s", flush=True)
    out = dict(
        source="oracle/ (eq. 9 component solves, eq. 19 combination + lift, adjoint), "
               "workloads.c3(L=10), written by tests/golden/make_c3_golden.py",
        pos_n=pos_n.tolist(), pos_m=pos_m.tolist(), pos_s=pos_s.tolist(),
        U=U_s.tolist(),
        df=df[pos_n, pos_m].tolist(), du0=du0[pos_s].tolist(), dv0=dv0[pos_s].tolist(),
        df_norm=float(np.linalg.norm(df)), du0_norm=float(np.linalg.norm(du0)),
        dv0_norm=float(np.linalg.norm(dv0)),
        components=comps)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {OUT} in {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
