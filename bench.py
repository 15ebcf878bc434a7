"""Benchmark: combined space-time DoFs/s of the sparse-grid wave solver.

Workload: d=2, Omega=(0,1)^2, L=10, c=1, T=1, manufactured
u = sin(pi x) sin(pi y) sin(pi t) (f = pi^2 u, u0 = 0, v0 = pi sin sin),
adjoint cotangent g ~ N(0,1) (seed 0); all synthetic, FP64, inputs resident
in HBM before timing.

A step is one pass of the whole hot path: forward (load restriction, 17
component solves, combination) and adjoint (restriction of g, transposed
solves, df/du0/dv0), replayed from one captured HIP graph (the batched form;
the adjoint on a branch concurrent with the forward, the cotangent being
given).  value = N_sparse DoFs per step / seconds per step.

Also reported (config): forward-only DoFs/s (eager and from a forward-only
graph), the per-component plain loop, fwd+adj/fwd, the per-stage times from
HIP events on the launch stream, and the 256-problem batch (d=2, L ~ U{6..10},
4x4 wave-speed blocks): its batched graph against the plain per-problem loop
and the roofline of its merged component solves.
"""

import argparse
import json
import math
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
    ap.add_argument("--cpu-max-dofs", type=int, default=40000,
                    help="largest component (DoFs) in the oracle's timed sample")
    ap.add_argument("--cpu-max-comps", type=int, default=6,
                    help="components in the oracle's timed sample (size-stratified)")
    ap.add_argument("--cpu-procs", type=int, default=8)
    ap.add_argument("--no-c5", action="store_true", help="skip the 256-problem batch")
    ap.add_argument("--c5-n", type=int, default=256)
    ap.add_argument("--c5-steps", type=int, default=3)
    ap.add_argument("--no-c5-plain", action="store_true",
                    help="skip the batch's plain per-component loop (profiling runs)")
    ap.add_argument("--no-1d", action="store_true", help="skip the two 1-D configurations")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of one fine array (counter scaling)")
    return ap.parse_args()


def _cpu_solve_phase(spec, data, comps, reps, barrier=None):
    """Warm the oracle's caches for `comps` (time and spatial matrices, cross
    operators, sparse LU factors: its assembly), then time `reps` passes of
    the solve phase (load of eq. 9, solve, prolongation), 1 BLAS thread.
    Returns (assembly seconds, list of pass seconds)."""
    from threadpoolctl import threadpool_limits

    from oracle import Problem
    with threadpool_limits(limits=1):
        prob = Problem(*spec.args())
        t0 = time.perf_counter()
        for jx, jt, s in comps:
            prob.prolong(jx, jt, prob.solve(jx, jt, prob.load(jx, jt, data["f"], data["u0"],
                                                               data["v0"])))
        t_asm = time.perf_counter() - t0
        times = []
        for _ in range(reps):
            if barrier is not None:
                barrier.wait()
            t0 = time.perf_counter()
            U = np.zeros((spec.nt(), spec.nx() ** spec.d))
            for jx, jt, s in comps:
                b = prob.load(jx, jt, data["f"], data["u0"], data["v0"])
                U += s * prob.prolong(jx, jt, prob.solve(jx, jt, b))
            times.append(time.perf_counter() - t0)
            if barrier is not None:
                barrier.wait()
    return t_asm, times


def _pool_worker(spec, data, comps, reps, barrier, q):
    q.put(_cpu_solve_phase(spec, data, comps, reps, barrier))


def _host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(spec, data, max_dofs, max_comps, procs, reps=3):
    """The oracle (plain FP64 CPU code) on a bounded sample of the same
    workload: up to max_comps components with at most max_dofs DoFs, spread
    evenly over the sizes (each load streams the whole fine array).  Assembly (its
    caches) is warmed first and reported apart; the solve phase (load +
    sparse LU solve with refinement + prolongation) is timed, median of
    `reps`, in one process and in a pool of `procs` processes that split the
    components by longest-processing-time on their DoFs (the component solves
    are independent).  Runs before the GPU is initialised (fork-safe)."""
    import multiprocessing as mp

    from oracle import levels
    size = lambda c: levels.n_space(c[0], spec.d) * levels.n_time(c[1])
    comps = sorted((c for c in levels.components(spec.L) if size(c) <= max_dofs), key=size)
    if len(comps) > max_comps:
        pick = np.linspace(0, len(comps) - 1, max_comps).round().astype(int)
        comps = [comps[i] for i in sorted(set(pick.tolist()))]
    dofs = sum(size(c) for c in comps)
    t_asm, times = _cpu_solve_phase(spec, data, comps, reps)
    t1 = float(np.median(times))
    # pool: longest-processing-time assignment of the components to workers
    P = max(1, min(procs, len(comps), os.cpu_count() or 1))
    parts = [[] for _ in range(P)]
    loads = [0] * P
    for c in sorted(comps, key=size, reverse=True):
        k = loads.index(min(loads))
        parts[k].append(c)
        loads[k] += size(c)
    ctx = mp.get_context("fork")
    barrier, q = ctx.Barrier(P), ctx.Queue()
    ws = [ctx.Process(target=_pool_worker, args=(spec, data, parts[k], reps, barrier, q))
          for k in range(P)]
    for w in ws:
        w.start()
    res = [q.get() for _ in ws]
    for w in ws:
        w.join()
    # pass r of the pool ends when its slowest worker does
    tP = float(np.median([max(r[1][i] for r in res) for i in range(reps)]))
    ncomp = len(levels.components(spec.L))
    return {"value": dofs / tP, "unit": "DoF/s", "cores": P, "kind": "oracle",
            "single_process_value": dofs / t1,
            "assembly_s": t_asm,
            "host": _host_info(),
            "sample": (f"solve phase (load + SuperLU solve with refinement + prolongation) of "
                       f"{len(comps)} of the {ncomp} components "
                       f"{' '.join(f'({c[0]},{c[1]})' for c in comps)}, size-stratified "
                       f"among those with <= {max_dofs} DoFs "
                       f"({dofs} DoFs) of the same d=2 L={spec.L} workload, caches warmed "
                       f"first (assembly {t_asm:.1f} s, not timed); median of {reps}; value: "
                       f"{P} single-threaded processes (LPT split, {tP:.2f} s); single "
                       f"process {t1:.2f} s")}


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
    """Energy of the last solution at K uniform instants.  In 2-D with
    16 x 16 tiles the element forms are applied inside the evaluation of
    u_h and d_t u_h over the instants (no field is written: the reads are
    the component solutions, u0 and the element speeds, and one partial sum
    per instant and tile is written)."""
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
    return {"instants": K, "ms": t * 1e3, "us_per_instant": t * 1e6 / K,
            "fine_nodes_evaluated_per_s": 2.0 * K * nspace / t,
            "E_first_last": [float(E[0]), float(E[-1])]}


def time_l2(sv, u0, stream, reps=3):
    """Relative L^2(Q_T) error of the manufactured solution u = sin(pi x)
    sin(pi y) sin(pi t) (the benchmark workload's exact solution) by the
    library's quadrature: u_h at 3 Gauss instants per finest time interval,
    2 x 2 Gauss points per finest element; the exact values at the points
    are generated on the device (separable)."""
    import torch
    sv.l2_setup()
    p = sv.l2_points()
    dev = u0.device
    st = torch.sin(math.pi * torch.from_numpy(p["t"]).to(dev))
    sx = torch.sin(math.pi * torch.from_numpy(p["xq"]).to(dev))
    sy = torch.sin(math.pi * torch.from_numpy(p["yq"]).to(dev))
    uq = st[:, None, None] * sy[None, :, None] * sx[None, None, :]
    with torch.cuda.stream(stream):
        out = sv.l2_error(u0, uq, stream=stream)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            sv.l2_error(u0, uq, out=out, stream=stream)
        e1.record(stream)
    stream.synchronize()
    err, nrm = (float(v) for v in out.cpu())
    res = {"relative_l2_error": math.sqrt(err / nrm), "norm_exact": math.sqrt(nrm),
           "ms": e0.elapsed_time(e1) / reps, "instants": int(p["t"].size),
           "points_per_instant": int(p["xq"].size) ** 2}
    del uq
    torch.cuda.empty_cache()
    return res


def coarse_mesh_study(sg, spec, sv, f, u0, v0, stream, b0s=(1, 2, 3), reps=3):
    """The coarse-mesh study of Sec. 6.3 (Fig. 10) on the benchmark workload:
    the same finest level with coarsest levels b0 (h_0 = 2^-b0): components,
    sparse DoFs, forward time (eager, after a warm-up) and the relative
    L^2(Q_T) error of the manufactured solution."""
    import torch
    U = torch.empty(sv.shape, dtype=torch.float64, device=u0.device)
    out = {}
    for b0 in b0s:
        svb = sv if b0 == 1 else sg.SparseGridWave(*spec.args(), tuned=True, b0=b0)
        with torch.cuda.stream(stream):
            svb.solve(f, u0, v0, out=U, stream=stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            for _ in range(reps):
                svb.solve(f, u0, v0, out=U, stream=stream)
            e1.record(stream)
        stream.synchronize()
        l2 = time_l2(svb, u0, stream, reps=1)
        out[str(b0)] = {"components": svb.n_components, "n_sparse": svb.n_sparse,
                        "forward_ms": e0.elapsed_time(e1) / reps,
                        "relative_l2_error": l2["relative_l2_error"]}
        if svb is not sv:
            svb.close()
    del U
    torch.cuda.empty_cache()
    return out


def configs_1d(sg, stream, reps=10):
    """The two 1-D configurations: c2 (L=12, T=2, c = 1 | 1/2, f = 0,
    Gaussian u0) and c4 (L=14, c on 8 cells ~ U[0.5, 2], Gaussian source,
    u0 = 0.1 sin(pi x); seeded N(0,1) cotangent).  Forward + adjoint replayed
    from one captured graph (adjoint on its concurrent branch): ms per step,
    sparse DoFs per second and the rate of the four fine-array passes
    (read f, write U, read g, write df) against 8 TB/s."""
    import numpy as np
    import torch
    import workloads
    out = {}
    for name, (spec, data) in (("c2", workloads.c2()), ("c4", workloads.c4())):
        dev = "cuda:0"
        to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        f, u0, v0 = to(data["f"]), to(data["u0"]), to(data["v0"])
        g = to(np.random.default_rng([0, 2000]).standard_normal(spec.shape()))
        sv = sg.SparseGridWave(*spec.args(), tuned=True)
        U = torch.empty(sv.shape, dtype=torch.float64, device=dev)
        df = torch.empty_like(U)
        du0 = torch.empty(sv.space_shape, dtype=torch.float64, device=dev)
        dv0 = torch.empty_like(du0)
        with torch.cuda.stream(stream):
            sv.capture(f, u0, v0, U, g, df, du0, dv0, stream=stream)
            sv.replay(stream=stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            for _ in range(reps):
                sv.replay(stream=stream)
            e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / reps
        fine_bytes = 8 * sv.n_full
        out[name] = {"spec": repr(spec), "n_sparse": sv.n_sparse, "n_full": sv.n_full,
                     "components": sv.n_components, "ms_per_step": ms,
                     "fwd_adj_dofs_per_s": sv.n_sparse / (ms * 1e-3),
                     "fine_pass_GB_per_s": 4 * fine_bytes / (ms * 1e-3) / 1e9,
                     "fine_pass_frac_of_hbm": 4 * fine_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        sv.close()
        del f, u0, v0, g, U, df, du0, dv0
        torch.cuda.empty_cache()
    return out


def _gaussians_on_device(spec, centres, dev, width=0.05):
    """The batch workload's source f (sum of space-time Gaussians with the
    given centres (x, y, t)) generated directly in device memory; each
    Gaussian is a product of 1-D factors."""
    import torch
    t = torch.arange(spec.nt(), dtype=torch.float64, device=dev) * (spec.T / 2 ** spec.J)
    x = torch.arange(1, 2 ** spec.J, dtype=torch.float64, device=dev) * (spec.lengths[0] / 2 ** spec.J)
    y = torch.arange(1, 2 ** spec.J, dtype=torch.float64, device=dev) * (spec.lengths[1] / 2 ** spec.J)
    f = torch.zeros(spec.shape(), dtype=torch.float64, device=dev)
    w2 = 2.0 * width * width
    for cx, cy, ct in centres:
        gt = torch.exp(-(t - ct) ** 2 / w2)
        gs = torch.exp(-(y - cy) ** 2 / w2)[:, None] * torch.exp(-(x - cx) ** 2 / w2)[None, :]
        f.add_(gt[:, None, None] * gs[None, :, :])
    return f


def c5_batch(args, stream):
    """The 256-problem batch (d=2, L ~ U{6..10}, 4x4 blocks of wave speed in
    [0.5, 2], f = three space-time Gaussians, u0 = v0 = 0).
    A step is the forward and the adjoint of every problem, replayed from one
    captured HIP graph (every stage, streaming or solve, one launch over all
    problems per kernel variant; the adjoint after the forward).  Three fine arrays per problem fit in HBM
    (3 x 68 GiB for the seed-0 draw): f, U and df; the timed cotangent is the
    source array itself (both directions only read it).  Parity of this
    workload, with an N(0,1) cotangent, is the business of the tests."""
    import torch

    import paper_2606_09688_amd as sg
    import workloads
    dev = "cuda:0"
    specs = workloads.c5_specs()[:args.c5_n]
    t0 = time.perf_counter()
    svs = [sg.SparseGridWave(*sp.args(), tuned=True) for sp in specs]
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = sg.SparseGridBatch(svs)
    t_merge = time.perf_counter() - t0
    n, n_sparse, table_bytes = batch.info()
    zeros, fs, Us, Ds, du0s, dv0s = {}, [], [], [], [], []
    for i, sp in enumerate(specs):
        fs.append(_gaussians_on_device(sp, workloads.c5_centres(i), dev))
        Us.append(torch.empty(sp.shape(), dtype=torch.float64, device=dev))
        Ds.append(torch.empty(sp.shape(), dtype=torch.float64, device=dev))
        zeros.setdefault(sp.L, torch.zeros(sp.space_shape(), dtype=torch.float64, device=dev))
        du0s.append(torch.empty(sp.space_shape(), dtype=torch.float64, device=dev))
        dv0s.append(torch.empty(sp.space_shape(), dtype=torch.float64, device=dev))
    u0s = [zeros[sp.L] for sp in specs]
    gs = fs  # the cotangent: read-only in both directions
    torch.cuda.synchronize()
    n_full = sum(sp.nt() * sp.nx() ** 2 for sp in specs)
    # eager batched pass with stage events (merged solve stages timed)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    batch.set_events(ev)
    with torch.cuda.stream(stream):
        for _ in range(2):
            batch.solve(fs, u0s, u0s, Us, stream=stream)
            batch.adjoint(gs, Ds, du0s, dv0s, stream=stream)
    stream.synchronize()
    el = lambda a, b: ev[a].elapsed_time(ev[b]) * 1e-3
    st = {"fwd": el(0, 3), "fwd_solves": el(1, 2), "adj": el(4, 7), "adj_solves": el(5, 6)}
    batch.set_events(None)
    # the captured graph: forward + adjoint of all problems
    with torch.cuda.stream(stream):
        batch.capture(fs, u0s, u0s, Us, gs, Ds, du0s, dv0s, stream=stream)
        batch.replay(stream=stream)
    stream.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(args.c5_steps):
            batch.replay(stream=stream)
    stream.synchronize()
    t_graph = (time.perf_counter() - t0) / args.c5_steps
    # plain loop: each problem's literal per-component forward, then its
    # adjoint, one problem after the other (host-driven launches, no graph)
    t_plain = float("nan")
    if not args.no_c5_plain:
        with torch.cuda.stream(stream):
            t0 = time.perf_counter()
            for sv, f, g, U, D, z, du, dv in zip(svs, fs, gs, Us, Ds, u0s, du0s, dv0s):
                sv.solve(f, z, z, out=U, plain=True, stream=stream)
                sv.adjoint(g, D, du, dv, stream=stream)
            stream.synchronize()
            t_plain = time.perf_counter() - t0
    # compulsory component I/O of one direction's solves (read the load,
    # write the solution) and the tables they read
    io = 16.0 * n_sparse
    t_solves = 0.5 * (st["fwd_solves"] + st["adj_solves"])
    ach_io = io / t_solves / 1e9
    ach_all = (io + table_bytes) / t_solves / 1e9
    counts = {}
    for sp in specs:
        counts[sp.L] = counts.get(sp.L, 0) + 1
    out = {
        "workload": (f"{n} problems d=2 Omega=(0,1)^2 T=1, L ~ U{{6..10}} (seed 0: "
                     + ", ".join(f"L={L}: {c}" for L, c in sorted(counts.items()))
                     + "), c on 4x4 blocks ~ U[0.5,2], f = 3 space-time Gaussians, u0=v0=0, "
                       "cotangent = f; step = forward + adjoint of all problems (one hipGraph)"),
        "n_sparse": n_sparse,
        "n_full": n_full,
        "assembly_s": t_asm,
        "batch_merge_s": t_merge,
        "ms_per_step": t_graph * 1e3,
        "batched_fwd_adj_dofs_per_s": n_sparse / t_graph,
        "plain_loop_ms_per_step": None if t_plain != t_plain else t_plain * 1e3,
        "batched_over_plain_speedup": None if t_plain != t_plain else t_plain / t_graph,
        "fine_array_GB_per_s": 4 * 8.0 * n_full / t_graph / 1e9,
        "eager_stage_ms": {k: v * 1e3 for k, v in st.items()},
        "solve_roofline": {
            "what": "merged component solves of one direction (mean of forward and adjoint)",
            "ms": t_solves * 1e3,
            "component_io_bytes": io,
            "table_bytes": table_bytes,
            "achieved_io_GB_per_s": ach_io,
            "achieved_with_tables_GB_per_s": ach_all,
            "peak": HBM_PEAK_GBS,
            "frac_io": ach_io / HBM_PEAK_GBS,
            "frac_with_tables": ach_all / HBM_PEAK_GBS,
        },
        "tuned": sg.tuning_status(),
    }
    del fs, gs, Us, Ds
    batch.close()
    for sv in svs:
        sv.close()
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import workloads
    spec, data = workloads.c3(L=args.L)
    # the oracle's CPU baseline runs first, before the GPU is initialised, so
    # that its process pool can fork
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, data, args.cpu_max_dofs, args.cpu_max_comps, args.cpu_procs)

    import torch

    import paper_2606_09688_amd as sg

    dev = "cuda:0"
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    f, u0, v0, g = (to(data[k]) for k in ("f", "u0", "v0", "g"))
    sv = sg.SparseGridWave(*spec.args(), tuned=True)
    U = torch.empty(sv.shape, dtype=torch.float64, device=dev)
    df = torch.empty(sv.shape, dtype=torch.float64, device=dev)
    du0 = torch.empty(sv.space_shape, dtype=torch.float64, device=dev)
    dv0 = torch.empty(sv.space_shape, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    nfull = sv.n_full

    # ---- batched: forward + adjoint in one captured graph ------------------
    # The step graph runs the adjoint on its own branch, concurrent with the
    # forward (the cotangent is given).  Kernel durations come from a second
    # capture with stage events set, which keeps the directions one after
    # the other so that every streaming kernel runs alone: event-record nodes
    # bracket the kernels inside that graph on the launch stream.  Its
    # warm-up replays bracket all four (their durations, and which one
    # dominates); its timed replays bracket the dominant kernel only (every
    # event node costs a replay a few microseconds).  Timed replays run back
    # to back (no host synchronisation between them).
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

    def timed_replays(k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(k):
                sv.replay(stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    graph_events = capture(ev)
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            sv.replay(stream=stream)
    stream.synchronize()
    dom = "restriction of f"
    t_step_seq = float("nan")
    if graph_events:
        kern_t = {k: ev[a].elapsed_time(ev[b]) * 1e-3 for k, (a, b) in kern_ev.items()}
        dom = max(kern_t, key=kern_t.get)
        ia, ib = kern_ev[dom]
        graph_events = capture([e if i in (ia, ib) else None for i, e in enumerate(ev)])
        with torch.cuda.stream(stream):
            sv.replay(stream=stream)
        stream.synchronize()
        t_step_seq = timed_replays(args.steps)
        if graph_events:
            kern_t[dom] = ev[ia].elapsed_time(ev[ib]) * 1e-3
    # the step graph (no events: the adjoint branch runs concurrently)
    capture(None)
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            sv.replay(stream=stream)
    stream.synchronize()
    t_step = timed_replays(args.steps)
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

    # ---- forward-only graph (the batched forward) ----------------------------
    sv.set_events(None)
    with torch.cuda.stream(stream):
        sv.capture(f, u0, v0, U, stream=stream)
        sv.replay(stream=stream)
    stream.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            sv.replay(stream=stream)
    stream.synchronize()
    t_graph_fwd = (time.perf_counter() - t0) / args.steps

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

    # ---- Sec. 6.3 diagnostics: energy at 800 instants (element forms inside
    # the evaluation over the instants) and the relative L^2(Q_T) error of the
    # manufactured solution by quadrature
    K_e = 800
    energy_out, l2_out = None, None
    if not args.no_energy:
        energy_out = time_energy(sv, u0, stream, spec.T, K_e, nfull // sv.shape[0])
        l2_out = time_l2(sv, u0, stream)
        l2_out["coarse_mesh_study"] = coarse_mesh_study(sg, spec, sv, f, u0, v0, stream)
    configs_out = None if args.no_1d else configs_1d(sg, stream)

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
            "sequential_graph_ms_per_step": t_step_seq * 1e3,
            "eager_fwd_dofs_per_s": ns / stage["fwd"],
            "graph_fwd_dofs_per_s": ns / t_graph_fwd,
            "plain_fwd_dofs_per_s": ns / t_plain,
            "graph_fwd_over_plain_fwd_speedup": t_plain / t_graph_fwd,
            "eager_fwd_over_plain_fwd_speedup": t_plain / stage["fwd"],
            "fwd_adj_over_fwd": (stage["fwd"] + stage["adj"]) / stage["fwd"],
            "plain_vs_fused_rel_l2": plain_diff,
            "graph_equals_eager": graph_equals_eager,
            "energy": energy_out,
            "l2_error": l2_out,
            "configs_1d": configs_out,
            "stage_ms": {k: v * 1e3 for k, v in stage.items()},
            "kernel_ms": {k: v * 1e3 for k, v in kern_t.items()},
            "kernel_ms_from": (f"{dom}: last timed replay of the graph with the directions in "
                               "sequence (kernels alone); the others: its last warm-up replay"
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
    out["config"]["tuned"] = sg.tuning_status()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    # ---- the 256-problem batch ----------------------------------------------
    if not args.no_c5:
        del f, g, U, df, du0, dv0
        sv.close()
        torch.cuda.empty_cache()
        out["config"]["batch_c5"] = c5_batch(args, stream)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
