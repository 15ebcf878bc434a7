"""Benchmark: combined space-time DoFs/s of the sparse-grid wave solver.

Workload: d=2, Omega=(0,1)^2, L=10, c=1, T=1, manufactured
u = sin(pi x) sin(pi y) sin(pi t) (f = pi^2 u, u0 = 0, v0 = pi sin sin),
adjoint cotangent g ~ N(0,1) (seed 0); all synthetic, FP64, inputs resident
in HBM before timing.

A step is one pass of the whole hot path: forward (load restriction, 17
component solves, combination) and adjoint (restriction of g, transposed
solves, df/du0/dv0), replayed from one captured HIP graph (the batched form).
value = N_sparse DoFs per step / seconds per step.

Also reported (config): forward-only DoFs/s, the per-component plain loop,
fwd+adj/fwd, and the per-stage times from HIP events on the launch stream.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "combined space–time DoFs/sec at d=2 L=10 (plain vs batched); fwd+adj/fwd"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=10)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true",
                    help="skip the energy diagnostic (counter runs of the streaming kernels)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of one fine array (counter scaling)")
    return ap.parse_args()


def cpu_baseline(spec, data, budget_s):
    """Time the oracle (forward: load, solve, prolongation per component) on
    the components of the same workload, smallest first, until the budget is
    used; single-threaded BLAS."""
    from threadpoolctl import threadpool_limits

    from oracle import Problem
    with threadpool_limits(limits=1):
        prob = Problem(*spec.args())
        order = sorted(prob.comps, key=lambda c: (2 ** c[0] - 1) ** spec.d * (2 ** c[1] + 1))
        dofs = 0
        done = []
        t0 = time.perf_counter()
        U = np.zeros((spec.nt(), (spec.nx()) ** spec.d))
        for jx, jt, s in order:
            b = prob.load(jx, jt, data["f"], data["u0"], data["v0"])
            u = prob.solve(jx, jt, b)
            U += s * prob.prolong(jx, jt, u)
            dofs += u.size
            done.append(f"({jx},{jt})")
            if time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    return {"value": dofs / el, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"forward load+solve+prolongation of {len(done)} of "
                       f"{len(prob.comps)} components {' '.join(done)} "
                       f"({dofs} DoFs, {el:.1f} s, smallest first, 1 BLAS thread)")}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c3_L10.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2606_09688_amd", "csrc", "kernels.hip")


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or the kernels changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def copy_calibration(args):
    """A plain device copy of one fine array (known bytes), for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    import paper_2606_09688_amd as sg
    spec, _ = __import__("workloads").c3(L=args.L, with_cotangent=False)
    n = spec.nt() * spec.nx() ** spec.d
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 8 * n, "bytes_written": 8 * n,
                                           "launches": 3, "library": sg.__name__}}), flush=True)


def time_energy(sv, u0, stream, T, K, nspace, reps=5):
    """Energy of the last solution at K uniform instants: two streaming
    prolongations over the instants and an element-wise reduction reading
    both fields back (4 K nspace doubles of algorithmic traffic)."""
    import torch
    sv.energy_setup(np.linspace(0.0, T, K))
    with torch.cuda.stream(stream):
        E = sv.energy(u0, stream=stream)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            sv.energy(u0, out=E, stream=stream)
        e1.record(stream)
    stream.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    nbytes = 4.0 * K * nspace * 8
    return {"instants": K, "ms": t * 1e3, "hbm_bytes": nbytes, "GB_per_s": nbytes / t / 1e9,
            "E_first_last": [float(E[0]), float(E[-1])]}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2606_09688_amd as sg
    import workloads

    dev = "cuda:0"
    spec, data = workloads.c3(L=args.L)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    f, u0, v0, g = (to(data[k]) for k in ("f", "u0", "v0", "g"))
    sv = sg.SparseGridWave(*spec.args())
    U = torch.empty(sv.shape, dtype=torch.float64, device=dev)
    df = torch.empty(sv.shape, dtype=torch.float64, device=dev)
    du0 = torch.empty(sv.space_shape, dtype=torch.float64, device=dev)
    dv0 = torch.empty(sv.space_shape, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    nfull = sv.n_full

    # ---- batched: forward + adjoint in one captured graph ------------------
    # Event-record nodes bracket streaming kernels inside the graph, so a
    # replay times its own kernels on the launch stream.  The warm-up replays
    # bracket all four (their durations, and which one dominates); the timed
    # graph brackets the dominant kernel only, since every event node costs
    # the replay a few microseconds.  The timed steps run back to back (no
    # host synchronisation between them); the dominant kernel's duration is
    # read after the final synchronisation, from the last timed replay.
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(15)]
    kern_ev = {"restriction of f": (1, 2), "prolongation into U": (5, 6),
               "restriction of g": (8, 9), "prolongation into df (mass stencil)": (12, 13)}
    kern_t = {k: 0.0 for k in kern_ev}

    def capture(events):
        sv.set_events(events)
        try:
            with torch.cuda.stream(stream):
                sv.capture(f, u0, v0, U, g, df, du0, dv0, stream=stream)
            return True
        except sg.SGError:
            sv.set_events(None)  # runtime without captured event records
            with torch.cuda.stream(stream):
                sv.capture(f, u0, v0, U, g, df, du0, dv0, stream=stream)
            return False

    graph_events = capture(ev)
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            sv.replay(stream=stream)
    stream.synchronize()
    dom = "restriction of f"
    if graph_events:
        kern_t = {k: ev[a].elapsed_time(ev[b]) * 1e-3 for k, (a, b) in kern_ev.items()}
        dom = max(kern_t, key=kern_t.get)
        ia, ib = kern_ev[dom]
        graph_events = capture([e if i in (ia, ib) else None for i, e in enumerate(ev)])
        with torch.cuda.stream(stream):
            sv.replay(stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            sv.replay(stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    if graph_events:
        kern_t[dom] = ev[ia].elapsed_time(ev[ib]) * 1e-3
    sv.set_events(ev)
    U_graph, df_graph = U.clone(), df.clone()

    # ---- eager runs with stage events (forward, adjoint) --------------------
    reps = max(3, args.steps // 2)
    stage = {k: 0.0 for k in ("fwd", "load_restrict", "solves", "combine", "adj",
                              "adj_restrict", "adj_solves", "df_prolong")}
    with torch.cuda.stream(stream):
        sv.solve(f, u0, v0, out=U, stream=stream)
        sv.adjoint(g, df, du0, dv0, stream=stream)
    stream.synchronize()
    for _ in range(reps):
        with torch.cuda.stream(stream):
            sv.solve(f, u0, v0, out=U, stream=stream)
            sv.adjoint(g, df, du0, dv0, stream=stream)
        stream.synchronize()
        el = lambda a, b: ev[a].elapsed_time(ev[b]) * 1e-3
        stage["fwd"] += el(0, 6)
        stage["load_restrict"] += el(1, 2)
        stage["solves"] += el(3, 4)
        stage["combine"] += el(5, 6)
        stage["adj"] += el(7, 14)
        stage["adj_restrict"] += el(8, 9)
        stage["adj_solves"] += el(10, 11)
        stage["df_prolong"] += el(12, 13)
    sv.set_events(None)
    stage = {k: v / reps for k, v in stage.items()}
    graph_equals_eager = bool(torch.equal(U_graph, U) and torch.equal(df_graph, df))
    del U_graph, df_graph

    # ---- plain per-component loop (forward) ---------------------------------
    t_plain, plain_diff = float("nan"), float("nan")
    if args.plain_steps > 0:
        Up = torch.empty_like(U)
        with torch.cuda.stream(stream):
            sv.solve(f, u0, v0, out=Up, plain=True, stream=stream)
        stream.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(args.plain_steps):
                sv.solve(f, u0, v0, out=Up, plain=True, stream=stream)
        stream.synchronize()
        t_plain = (time.perf_counter() - t0) / args.plain_steps
        plain_diff = float((Up - U).norm() / U.norm())
        del Up

    # ---- energy of the solution at 800 instants (Sec. 6.3 diagnostic) ------
    # two streaming prolongations over the instants (value and time
    # derivative of u_h) and an element-wise reduction that reads both back
    K_e = 800
    energy_out = None
    if not args.no_energy:
        energy_out = time_energy(sv, u0, stream, spec.T, K_e, nfull // sv.shape[0])

    # dominant fine-grid kernel (timed inside the last timed graph replay when
    # the runtime records captured events, else in the eager runs): each
    # streams 8 bytes per fine-grid value
    eager_t = {"restriction of f": stage["load_restrict"],
               "prolongation into U": stage["combine"],
               "restriction of g": stage["adj_restrict"],
               "prolongation into df (mass stencil)": stage["df_prolong"]}
    if graph_events and not all(0.5 < kern_t[k] / eager_t[k] < 2.0 for k in kern_t):
        graph_events = False  # event nodes did not bracket the kernels
    if not graph_events:
        kern_t = eager_t
    name = max(kern_t, key=kern_t.get)
    bytes_alg = 8.0 * nfull
    achieved = bytes_alg / kern_t[name] / 1e9
    ns = sv.n_sparse
    out = {
        "metric": METRIC,
        "value": ns / t_step,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"d=2 Omega=(0,1)^2 L={args.L} c=1 T=1, u=sin(pi x)sin(pi y)sin(pi t), "
                         "g~N(0,1) seed 0; step = forward + adjoint (hipGraph)"),
            "n_sparse": ns,
            "n_full": nfull,
            "batched_fwd_adj_dofs_per_s": ns / t_step,
            "eager_fwd_dofs_per_s": ns / stage["fwd"],
            "plain_fwd_dofs_per_s": ns / t_plain,
            "batched_fwd_over_plain_fwd_speedup": t_plain / stage["fwd"],
            "fwd_adj_over_fwd": (stage["fwd"] + stage["adj"]) / stage["fwd"],
            "plain_vs_fused_rel_l2": plain_diff,
            "graph_equals_eager": graph_equals_eager,
            "energy": energy_out,
            "stage_ms": {k: v * 1e3 for k, v in stage.items()},
            "kernel_ms": {k: v * 1e3 for k, v in kern_t.items()},
            "kernel_ms_from": (f"{dom}: last timed graph replay; the others: last warm-up replay"
                               if graph_events else "eager runs"),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": name,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(name),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, data, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
