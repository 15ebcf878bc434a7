"""Write full-array parity sketches of the oracle at full size.

Each output array X of the oracle is stored as its l2 norm and 16 separable
random projections (``workloads.sketch``); a test projects the library's
array the same way, and the root mean square of the differences estimates
the whole-array relative l2 error (an error confined to one time slab or
one tile changes the projections as much as one spread everywhere).

Workloads (all values from ``oracle/``: eq. (9) component solves, eq. (19)
combination + lift, and the transposed map):
  c3   d=2 L=10 manufactured sine problem, forward U and adjoint of g ~ N(0,1);
       every component's load and solution as well.
  c4   d=1 L=14 differentiation workload: U at the gradient point, and the
       adjoint of a seeded N(0,1) cotangent (workloads.c4_cotangent), with
       du0 and dv0 stored in full.
  c5   a stratified subset of the 256-problem batch (the first two problems
       of every level L = 6..10): U and the adjoint of its cotangent.

Usage:  python tests/golden/make_sketch_golden.py c3|c4|c5   (c3: ~10 min;
        c4: ~5 min; c5: ~25 min and ~20 GB RAM)
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

NPROJ = 16


def _entry(X):
    return {"norm": float(np.linalg.norm(X)), "sketch": workloads.sketch(X, NPROJ)}


def run_c3():
    t0 = time.perf_counter()
    spec, data = workloads.c3(L=10)
    prob = Problem(*spec.args())
    nt, n = spec.nt(), spec.nx()
    f, u0, v0 = data["f"], data["u0"], data["v0"]
    comps = []
    sols = []
    for jx, jt, s in prob.comps:
        b = prob.load(jx, jt, f, u0, v0)
        u = prob.solve(jx, jt, b)
        sols.append(u)
        na = 2 ** jx - 1
        comps.append(dict(jx=jx, jt=jt, sign=s, load=_entry(b.reshape(-1, na, na)),
                          sol=_entry(u.reshape(-1, na, na))))
        print(f"component ({jx},{jt}) {time.perf_counter() - t0:.0f} s", flush=True)
    U = prob.combine(sols, u0).reshape(nt, n, n)
    out = dict(U=_entry(U))
    del U
    df, du0, dv0 = prob.adjoint(data["g"])
    out.update(df=_entry(df.reshape(nt, n, n)), du0=_entry(du0.reshape(n, n)),
               dv0=_entry(dv0.reshape(n, n)), components=comps)
    return out, "workloads.c3(L=10)"


def run_c4():
    spec, data = workloads.c4()
    prob = Problem(*spec.args())
    U = prob.forward(data["f"], data["u0"], data["v0"])
    g = workloads.c4_cotangent(spec)
    df, du0, dv0 = prob.adjoint(g)
    out = dict(U=_entry(U), df=_entry(df), du0=_entry(du0), dv0=_entry(dv0),
               du0_full=du0.tolist(), dv0_full=dv0.tolist())
    return out, "workloads.c4() at the gradient point; adjoint of workloads.c4_cotangent"


def run_c5():
    specs = workloads.c5_specs()
    picks = []
    for L in range(6, 11):
        picks += [i for i, s in enumerate(specs) if s.L == L][:2]
    probs = []
    t0 = time.perf_counter()
    for i in picks:
        spec = specs[i]
        data = workloads.c5_data(spec, i)
        prob = Problem(*spec.args())
        U = prob.forward(data["f"], data["u0"], data["v0"]).reshape(spec.shape())
        df, du0, dv0 = prob.adjoint(data["g"])
        probs.append(dict(index=i, L=spec.L, U=_entry(U), df=_entry(df.reshape(spec.shape())),
                          du0=_entry(du0.reshape(spec.space_shape())),
                          dv0=_entry(dv0.reshape(spec.space_shape()))))
        print(f"problem {i} (L={spec.L}) {time.perf_counter() - t0:.0f} s", flush=True)
    return dict(problems=probs), "workloads.c5_specs() / c5_data(), first two problems per L"


def main():
    which = sys.argv[1]
    fn = {"c3": run_c3, "c4": run_c4, "c5": run_c5}[which]
    out, what = fn()
    out["source"] = (f"oracle/ forward (eq. 9, eq. 19 + lift) and adjoint; {what}; "
                     f"{NPROJ} separable projections (workloads.sketch); "
                     "written by tests/golden/make_sketch_golden.py")
    path = os.path.join(HERE, f"{which}_sketch.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
