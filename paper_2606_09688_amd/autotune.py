"""Launch-shape and tile autotuner with a JSON cache keyed by device.

The library reads a few tuning knobs from the environment when a problem is
assembled (sg_assemble); each selects a launch shape or a tile of one kernel
family:

  SG_RESTR_WG   resident workgroups per CU that size the grid of the
                streaming data restriction (2, 3, 4)
  SG_PROL_WG    the same for the prolongation into U
  SG_PROLM_WG   the same for the prolongation through the mass stencil (df)
  SG_GEMM_FOLD  folded sine transforms: 0 none, 1 x, 2 x and y of levels
                >= 7, 3 all (constant wave speed)
  SG_FDM_LEVEL  lowest spatial level of the 2-D variable-speed strip solver
                (3 .. 6; below it the dense pencils)
  SG_FDM_CH     rows per register chunk of the strip solver's tridiagonal
                sweeps (4, 8, 16)

A shape class is (d, L, constant or variable speed).  tune_class() times the
forward + adjoint of a representative seeded problem of the class for every
candidate value of one knob at a time, starting from the library defaults
(coordinate descent), keeps the fastest, and records the chosen values with
their times.  The cache is a JSON file
    {device key: {class key: {"knobs": {...}, "ms": t, "default_ms": t0}}}
with the device key "<gfx architecture>|<compute units>cu".
The committed cache (tuning/tiles.json) holds the results of a run on an
MI355X; SG_TUNING_CACHE names another file to read and write.

Usage (on the GPU):  python -m paper_2606_09688_amd.autotune d2-L10-c d2-L8-v ...
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning", "tiles.json")

KNOBS = {
    "SG_RESTR_WG": (2, 3, 4),
    "SG_PROL_WG": (2, 3, 4),
    "SG_PROLM_WG": (2, 3, 4),
    "SG_GEMM_FOLD": (0, 1, 2, 3),
    "SG_FDM_LEVEL": (3, 4, 5, 6),
    "SG_FDM_CH": (4, 8, 16),
}
DEFAULTS = {"SG_RESTR_WG": 3, "SG_PROL_WG": 3, "SG_PROLM_WG": 3, "SG_GEMM_FOLD": 2,
            "SG_FDM_LEVEL": 6, "SG_FDM_CH": 8}
CONST_ONLY = ("SG_GEMM_FOLD",)
VAR2_ONLY = ("SG_FDM_LEVEL", "SG_FDM_CH")

_status = {"device": None, "cache": None, "hits": [], "misses": []}


def cache_path():
    return os.environ.get("SG_TUNING_CACHE", DEFAULT_CACHE)


def device_key():
    """Architecture and compute-unit count (the marketing name is not a
    stable key: it is empty where the amdgpu device-name table is missing)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or ""
    return f"{arch.split(':')[0]}|{p.multi_processor_count}cu"


def class_key(d, L, const_c):
    return f"d{int(d)}-L{int(L)}-{'c' if const_c else 'v'}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(d, L, const_c):
    """Tuned knob values of the class on this device, or None."""
    key = class_key(d, L, const_c)
    dev = device_key()
    ent = _load(cache_path()).get(dev, {}).get(key)
    _status["device"] = dev
    _status["cache"] = cache_path()
    (_status["hits"] if ent else _status["misses"]).append(key)
    return None if ent is None else dict(ent["knobs"])


def status():
    """Which classes this process found in the cache (for reports)."""
    return {"device": _status["device"], "cache": _status["cache"],
            "hits": sorted(set(_status["hits"])), "misses": sorted(set(_status["misses"]))}


class knobs_set:
    """Context manager: the given knobs in the environment, restored after."""

    def __init__(self, knobs):
        self.knobs = knobs or {}
        self.saved = {}

    def __enter__(self):
        for k, v in self.knobs.items():
            self.saved[k] = os.environ.get(k)
            os.environ[k] = str(v)
        return self

    def __exit__(self, *exc):
        for k, v in self.saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


class _Shape:
    """A representative problem of a class: unit domain, T = 1, constant c or
    seeded speeds on 8 cells (1-D) / 4 x 4 blocks (2-D) in [0.5, 2]."""

    def __init__(self, d, L, const_c):
        import numpy as np
        self.d, self.L = d, L
        ncell = 1 if const_c else (8 if d == 1 else 4)
        self.args = (d, [1.0] * d, [ncell] * d,
                     [1.0] if const_c else list(np.random.default_rng(1).uniform(0.5, 2.0,
                                                                                  ncell ** d)),
                     1.0, L)
        n = 2 ** (L - 1) - 1
        self.space = (n,) * d
        self.full = (2 ** (L - 1) + 1,) + self.space


def _time_config(spec, knobs, data, reps=5):
    import torch

    from .binding import SparseGridWave
    with knobs_set(knobs):
        sv = SparseGridWave(*spec.args)
    f, u0, v0, g = data
    U = torch.empty_like(f)
    df = torch.empty_like(f)
    du0 = torch.empty_like(u0)
    dv0 = torch.empty_like(u0)
    for _ in range(2):
        sv.solve(f, u0, v0, out=U)
        sv.adjoint(g, df, du0, dv0)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sv.solve(f, u0, v0, out=U)
        sv.adjoint(g, df, du0, dv0)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    sv.close()
    ts.sort()
    return ts[len(ts) // 2]


def tune_class(d, L, const_c, log=print):
    """Coordinate descent over the knobs that apply to the class; returns
    the cache entry."""
    import torch
    spec = _Shape(d, L, const_c)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(1234)
    rnd = lambda shp: torch.randn(shp, generator=gen, dtype=torch.float64, device="cuda:0")
    data = (rnd(spec.full), rnd(spec.space), rnd(spec.space), rnd(spec.full))
    names = [k for k in KNOBS
             if not (k in CONST_ONLY and not const_c)
             and not (k in VAR2_ONLY and (const_c or d != 2))]
    best = {k: DEFAULTS[k] for k in names}
    t_def = _time_config(spec, best, data)
    t_best = t_def
    log(f"{class_key(d, L, const_c)}: defaults {t_def:.3f} ms")
    for k in names:
        for v in KNOBS[k]:
            if v == best[k]:
                continue
            trial = dict(best, **{k: v})
            t = _time_config(spec, trial, data)
            log(f"  {k}={v}: {t:.3f} ms")
            if t < 0.98 * t_best:  # keep a change only if it is clearly faster
                best, t_best = trial, t
    return {"knobs": best, "ms": t_best, "default_ms": t_def,
            "what": "median of 5 eager forward + adjoint passes, coordinate descent"}


def main(argv):
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("autotuning needs the GPU")
    path = cache_path()
    cache = _load(path)
    dev = device_key()
    for key in argv:
        d = int(key.split("-")[0][1:])
        L = int(key.split("-")[1][1:])
        const_c = key.endswith("-c")
        t0 = time.perf_counter()
        ent = tune_class(d, L, const_c, log=lambda m: print(m, flush=True))
        cache.setdefault(dev, {})[class_key(d, L, const_c)] = ent
        print(f"{key}: {ent['knobs']} {ent['ms']:.3f} ms (defaults {ent['default_ms']:.3f} ms), "
              f"tuned in {time.perf_counter() - t0:.0f} s", flush=True)
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
