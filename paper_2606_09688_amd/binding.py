"""ctypes binding of libsgwave.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors to device pointers and the current HIP stream to a stream handle.
There is no CPU fallback: if the shared library is missing or the tensors are
not FP64 device tensors, the calls raise.
"""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgwave.so")

SG_OK = 0
_STATUS = {0: "SG_OK", -1: "SG_EINVAL", -2: "SG_ENOMEM", -3: "SG_EDEVICE",
           -4: "SG_ENOTSUP", -5: "SG_ESTATE"}

_lib = None

_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int)
_c_llp = ctypes.POINTER(ctypes.c_longlong)

# name -> (restype, argtypes); mirrors include/sgwave.h
SIGNATURES = {
    "sg_assemble": (ctypes.c_int, [ctypes.c_int, _c_dp, _c_ip, _c_dp, ctypes.c_double,
                                   ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "sg_assemble_offset": (ctypes.c_int, [ctypes.c_int, _c_dp, _c_ip, _c_dp, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "sg_host_time_chunks": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_ip, _c_ip, _c_ip,
                                           _c_ip]),
    "sg_solve": (ctypes.c_int, [ctypes.c_void_p] * 6),
    "sg_solve_plain": (ctypes.c_int, [ctypes.c_void_p] * 6),
    "sg_solve_static": (ctypes.c_int, [ctypes.c_void_p] * 6),
    "sg_adjoint": (ctypes.c_int, [ctypes.c_void_p] * 6),
    "sg_graph_capture": (ctypes.c_int, [ctypes.c_void_p] * 10),
    "sg_graph_launch": (ctypes.c_int, [ctypes.c_void_p] * 2),
    "sg_query": (ctypes.c_int, [ctypes.c_void_p, _c_ip, _c_ip, _c_llp, _c_llp, _c_ip]),
    "sg_component_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_ip, _c_ip,
                                         _c_ip, _c_ip, _c_ip]),
    "sg_component_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_dp]),
    "sg_host_time_level": (ctypes.c_int, [ctypes.c_int, ctypes.c_double] + [_c_dp] * 7),
    "sg_host_taps": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, _c_ip, _c_dp]),
    "sg_host_pencil": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, _c_dp,
                                      _c_dp, _c_dp]),
    "sg_host_pencil_2d": (ctypes.c_int, [ctypes.c_int, _c_dp, _c_ip, _c_dp, _c_dp, _c_dp]),
    "sg_host_time_fdm": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, _c_ip] + [_c_dp] * 5),
    "sg_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "sg_batch_capture": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_void_p)] * 8
                         + [ctypes.c_void_p]),
    "sg_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sg_batch_info": (ctypes.c_int, [ctypes.c_void_p, _c_ip, _c_llp, _c_llp]),
    "sg_batch_set_events": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.c_int]),
    "sg_batch_solve": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_void_p)] * 4
                       + [ctypes.c_void_p]),
    "sg_batch_adjoint": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_void_p)] * 4
                         + [ctypes.c_void_p]),
    "sg_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sg_set_events": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.c_int]),
    "sg_energy_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_dp]),
    "sg_energy": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "sg_l2_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), _c_dp, _c_dp,
                                    ctypes.POINTER(ctypes.c_int), _c_dp, _c_dp]),
    "sg_l2_setup": (ctypes.c_int, [ctypes.c_void_p]),
    "sg_l2_error": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "sg_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sg_last_error": (ctypes.c_char_p, []),
}


class SGError(RuntimeError):
    pass


def lib():
    """Load libsgwave.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2606_09688_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, what):
    if status != SG_OK:
        msg = lib().sg_last_error().decode(errors="replace")
        raise SGError(f"{what} failed with {_STATUS.get(status, status)}: {msg}")


def _ptr(t, shape, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def host_time_level(b, T):
    """Dict of A, Alo, B, Blo (banded), Dlo, Dhi, g of level b (host introspection)."""
    import numpy as np
    nq = 2 ** b + 1
    out = {k: np.zeros((nq, 5)) for k in ("A", "Alo", "B", "Blo")}
    out.update({k: np.zeros(nq) for k in ("Dlo", "Dhi", "g")})
    dp = lambda a: a.ctypes.data_as(_c_dp)
    check(lib().sg_host_time_level(b, float(T), *[dp(out[k]) for k in
                                                 ("A", "Alo", "B", "Blo", "Dlo", "Dhi", "g")]),
          "sg_host_time_level")
    return out


def host_taps(kind, b, J, T):
    """(q0, w) tap table (kind 0: P1 load taps, 1: spline taps)."""
    import numpy as np
    n = 2 ** J + 1
    q0 = np.zeros(n, dtype=np.int32)
    w = np.zeros((n, 3))
    check(lib().sg_host_taps(kind, b, J, float(T), q0.ctypes.data_as(_c_ip),
                             w.ctypes.data_as(_c_dp)), "sg_host_taps")
    return q0, w


def host_time_chunks(q0, chunk):
    """(chunk, phase, nchunk) of a streaming pass whose finest-level window
    is q0 (sg_host_time_chunks)."""
    import numpy as np
    q = np.ascontiguousarray(q0, dtype=np.int32)
    out = [ctypes.c_int() for _ in range(3)]
    check(lib().sg_host_time_chunks(int(q.size), int(chunk), q.ctypes.data_as(_c_ip),
                                    *[ctypes.byref(o) for o in out]), "sg_host_time_chunks")
    return tuple(o.value for o in out)


def host_time_fdm(b, T):
    """Diagonalisation tables of time level b (sg_host_time_fdm): dict of
    lam (nu,), fin, ain (nu, nq), fout, aout (nq, nu), complex."""
    import numpy as np
    nq = 2 ** b + 1
    nu = ctypes.c_int()
    bufs = {k: np.zeros(2 * nq * nq) for k in ("lam", "fin", "fout", "ain", "aout")}
    dp = lambda a: a.ctypes.data_as(_c_dp)
    check(lib().sg_host_time_fdm(b, float(T), ctypes.byref(nu),
                                 *[dp(bufs[k]) for k in ("lam", "fin", "fout", "ain", "aout")]),
          "sg_host_time_fdm")
    u = nu.value
    c = lambda a, n: (a[0:2 * n:2] + 1j * a[1:2 * n:2])
    return {"lam": c(bufs["lam"], u),
            "fin": c(bufs["fin"], u * nq).reshape(u, nq),
            "ain": c(bufs["ain"], u * nq).reshape(u, nq),
            "fout": c(bufs["fout"], nq * u).reshape(nq, u),
            "aout": c(bufs["aout"], nq * u).reshape(nq, u)}


def host_pencil_2d(a, lengths, ncell, c_vals):
    """(K, M): dense level-a Q1 pencil in 2-D (n^2 x n^2, x fastest), c
    piecewise constant on ncell[0] x ncell[1] uniform blocks."""
    import numpy as np
    ln = np.ascontiguousarray(lengths, dtype=np.float64)
    nc = np.ascontiguousarray(ncell, dtype=np.int32)
    c = np.ascontiguousarray(c_vals, dtype=np.float64)
    n2 = (2 ** a - 1) ** 2
    K = np.zeros((n2, n2))
    M = np.zeros((n2, n2))
    check(lib().sg_host_pencil_2d(a, ln.ctypes.data_as(_c_dp), nc.ctypes.data_as(_c_ip),
                                  c.ctypes.data_as(_c_dp), K.ctypes.data_as(_c_dp),
                                  M.ctypes.data_as(_c_dp)), "sg_host_pencil_2d")
    return K, M


def host_pencil(a, length, c_vals):
    """(V, lam): M-orthonormal eigenpairs of the level-a P1 pencil (K(c), M)
    on (0, length), c piecewise constant on len(c_vals) uniform blocks."""
    import numpy as np
    c = np.ascontiguousarray(c_vals, dtype=np.float64)
    n = 2 ** a - 1
    V = np.zeros((n, n))
    lam = np.zeros(n)
    check(lib().sg_host_pencil(a, float(length), len(c), c.ctypes.data_as(_c_dp),
                               V.ctypes.data_as(_c_dp), lam.ctypes.data_as(_c_dp)),
          "sg_host_pencil")
    return V, lam


class SparseGridWave:
    """One assembled problem (sg_assemble) bound to the current HIP device.

    d: 1 or 2; lengths: side lengths; ncell: wave-speed blocks per axis;
    c_vals: block speeds (x fastest); T: final time; L: sparse level;
    b0: coarsest level of the combination (h_0 = 2^-b0, sg_assemble_offset).
    Arrays: f, U, g, df have shape (nt, n) / (nt, n, n); u0, v0 shape (n,) / (n, n).
    """

    def __init__(self, d, lengths, ncell, c_vals, T, L, tuned=False, b0=1):
        """tuned: build with the launch shapes the autotuner chose for this
        shape class on this device (autotune.lookup; library defaults if the
        class is not in the cache)."""
        import numpy as np
        L_ = lib()
        self.d = int(d)
        ln = (ctypes.c_double * d)(*[float(v) for v in lengths])
        nc = (ctypes.c_int * d)(*[int(v) for v in ncell])
        cv = np.ascontiguousarray(np.asarray(c_vals, dtype=np.float64).reshape(-1))
        knobs = None
        if tuned:
            from . import autotune
            knobs = autotune.lookup(d, L, bool(np.all(cv == cv[0])))
        h = ctypes.c_void_p()
        from .autotune import knobs_set
        with knobs_set(knobs):
            check(L_.sg_assemble_offset(d, ln, nc, cv.ctypes.data_as(_c_dp), float(T), int(L),
                                        int(b0), ctypes.byref(h)), "sg_assemble_offset")
        self._h = h
        nt, n, nc_ = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ns, nf = ctypes.c_longlong(), ctypes.c_longlong()
        check(L_.sg_query(h, ctypes.byref(nt), ctypes.byref(n), ctypes.byref(ns),
                          ctypes.byref(nf), ctypes.byref(nc_)), "sg_query")
        self.nt, self.n = nt.value, n.value
        self.n_sparse, self.n_full = ns.value, nf.value
        self.n_components = nc_.value
        self.space_shape = (self.n,) * self.d
        self.shape = (self.nt,) + self.space_shape
        self.T = float(T)
        self.L = int(L)
        self.b0 = int(b0)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.sg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- components -----------------------------------------------------
    def components(self):
        out = []
        for c in range(self.n_components):
            v = [ctypes.c_int() for _ in range(5)]
            check(lib().sg_component_info(self._h, c, *[ctypes.byref(x) for x in v]),
                  "sg_component_info")
            out.append(tuple(x.value for x in v))  # (jx, jt, sign, n_space, n_time)
        return out

    def component(self, c, stage):
        """Host copy of component c after the last solve (0: RHS, 1: solution)."""
        import numpy as np
        jx, jt, s, nsp, nq = self.components()[c]
        out = np.zeros((nq, nsp))
        check(lib().sg_component_copy(self._h, c, stage, out.ctypes.data_as(_c_dp)),
              "sg_component_copy")
        return out

    # ---- solves ---------------------------------------------------------
    def solve(self, f, u0, v0, out=None, plain=False, static=False, stream=None):
        """Forward solve into `out` (allocated if None).  plain: the literal
        per-component loop (sg_solve_plain); static: the fused path with the
        static device scratch (sg_solve_static)."""
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=f.device)
        fn = (lib().sg_solve_plain if plain else
              lib().sg_solve_static if static else lib().sg_solve)
        check(fn(self._h, _ptr(f, self.shape, "f"), _ptr(u0, self.space_shape, "u0"),
                 _ptr(v0, self.space_shape, "v0"), _ptr(out, self.shape, "U"),
                 _stream(stream)), "sg_solve")
        return out

    def adjoint(self, g, df=None, du0=None, dv0=None, want=(True, True, True), stream=None):
        dev = g.device
        if df is None and want[0]:
            df = torch.empty(self.shape, dtype=torch.float64, device=dev)
        if du0 is None and want[1]:
            du0 = torch.empty(self.space_shape, dtype=torch.float64, device=dev)
        if dv0 is None and want[2]:
            dv0 = torch.empty(self.space_shape, dtype=torch.float64, device=dev)
        check(lib().sg_adjoint(self._h, _ptr(g, self.shape, "g"),
                               _ptr(df, self.shape, "df", True),
                               _ptr(du0, self.space_shape, "du0", True),
                               _ptr(dv0, self.space_shape, "dv0", True), _stream(stream)),
              "sg_adjoint")
        return df, du0, dv0

    def capture(self, f, u0, v0, U, g=None, df=None, du0=None, dv0=None, stream=None):
        """Capture forward (+ adjoint when g is given) into a HIP graph.  The
        graph holds the tensors' device addresses, so they are kept alive
        here until the next capture or the solver's end."""
        s = stream if stream is not None else torch.cuda.current_stream()
        self._keep = (f, u0, v0, U, g, df, du0, dv0)
        check(lib().sg_graph_capture(
            self._h, _ptr(f, self.shape, "f"), _ptr(u0, self.space_shape, "u0"),
            _ptr(v0, self.space_shape, "v0"), _ptr(U, self.shape, "U"),
            _ptr(g, self.shape, "g", True), _ptr(df, self.shape, "df", True),
            _ptr(du0, self.space_shape, "du0", True),
            _ptr(dv0, self.space_shape, "dv0", True), _stream(s)), "sg_graph_capture")

    def energy_setup(self, times):
        """Prepare sg_energy at the given instants (ascending, in [0, T], no two
        consecutive ones more than one finest time interval apart)."""
        t = np.ascontiguousarray(np.asarray(times, dtype=np.float64).ravel())
        check(lib().sg_energy_setup(self._h, int(t.size), t.ctypes.data_as(_c_dp)),
              "sg_energy_setup")
        self._energy_k = int(t.size)

    def energy(self, u0, out=None, stream=None):
        """E(t_k) = 1/2 ||d_t u_h||^2 + 1/2 ||c grad u_h||^2 at the instants of
        energy_setup, for u_h the lifted solution of the last solve (u0 as given
        to it)."""
        k = getattr(self, "_energy_k", 0)
        if out is None:
            out = torch.empty(max(k, 1), dtype=torch.float64, device=u0.device)[:k]
        check(lib().sg_energy(self._h, _ptr(u0, self.space_shape, "u0"), _ptr(out, (k,), "E"),
                              _stream(stream)), "sg_energy")
        return out

    def l2_points(self):
        """The L^2(Q_T) quadrature rule: dict of t, wt (instants and weights)
        and the per-axis points xq (and yq in 2-D)."""
        K, nq = ctypes.c_int(0), ctypes.c_int(0)
        check(lib().sg_l2_points(self._h, ctypes.byref(K), None, None, ctypes.byref(nq), None,
                                 None), "sg_l2_points")
        t, wt = np.empty(K.value), np.empty(K.value)
        xq = np.empty(nq.value)
        yq = np.empty(nq.value) if self.d == 2 else None
        check(lib().sg_l2_points(self._h, None, t.ctypes.data_as(_c_dp), wt.ctypes.data_as(_c_dp),
                                 None, xq.ctypes.data_as(_c_dp),
                                 yq.ctypes.data_as(_c_dp) if yq is not None else None),
              "sg_l2_points")
        out = {"t": t, "wt": wt, "xq": xq}
        if yq is not None:
            out["yq"] = yq
        return out

    def l2_setup(self):
        """Prepare sg_l2_error (evaluation tables and workspace)."""
        check(lib().sg_l2_setup(self._h), "sg_l2_setup")
        self._l2_ready = True

    def l2_error(self, u0, uq, out=None, stream=None):
        """(int (u - u_h)^2, int u^2) over Q_T by the library's quadrature,
        uq the exact solution at the points of l2_points ([K][nq] or
        [K][nq][nq]); u_h the lifted solution of the last solve."""
        pts = self.l2_points()
        shape = (pts["t"].size,) + (pts["xq"].size,) * self.d
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=u0.device)
        check(lib().sg_l2_error(self._h, _ptr(u0, self.space_shape, "u0"), _ptr(uq, shape, "uq"),
                                _ptr(out, (2,), "out"), _stream(stream)), "sg_l2_error")
        return out

    def set_events(self, events):
        """Record the SG_NUM_EVENTS stage events (torch.cuda.Event list, None
        entries leave their point out) or None."""
        if events is None:
            check(lib().sg_set_events(self._h, None, 0), "sg_set_events")
            return
        for e in events:      # torch creates the underlying event on first record
            if e is not None and not e.cuda_event:
                e.record()
        torch.cuda.synchronize()
        arr = (ctypes.c_void_p * len(events))(
            *[e.cuda_event if e is not None else None for e in events])
        check(lib().sg_set_events(self._h, arr, len(events)), "sg_set_events")

    def replay(self, stream=None):
        check(lib().sg_graph_launch(self._h, _stream(stream)), "sg_graph_launch")


class SparseGridBatch:
    """Independent problems (any mix of d, L, speeds) run together
    (sg_batch_*): every stage (streaming or solve) one launch over all
    problems; eager (solve, adjoint) or
    captured into one HIP graph (capture, replay).  The solvers must stay
    alive while the batch exists."""

    def __init__(self, solvers):
        self._solvers = list(solvers)
        n = len(self._solvers)
        arr = (ctypes.c_void_p * n)(*[s._h for s in self._solvers])
        h = ctypes.c_void_p()
        check(lib().sg_batch_create(n, arr, ctypes.byref(h)), "sg_batch_create")
        self._h = h
        self._keep = None

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().sg_batch_destroy(h)
            self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, lst, space, name, allow_none=False):
        if lst is None:
            return None
        n = len(self._solvers)
        if len(lst) != n:
            raise ValueError(f"{name} needs one entry per problem")
        shapes = [s.space_shape if space else s.shape for s in self._solvers]
        out = [_ptr(t, shp, f"{name}[{i}]", allow_none)
               for i, (t, shp) in enumerate(zip(lst, shapes))]
        return (ctypes.c_void_p * n)(*[None if v is None else v.value for v in out])

    def info(self):
        """(number of problems, sum of component dimensions, bytes of tables
        read by one direction's merged solve stages)."""
        n, ns, tb = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_longlong()
        check(lib().sg_batch_info(self._h, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(tb)),
              "sg_batch_info")
        return n.value, ns.value, tb.value

    def set_events(self, events):
        """Stage events of the eager batched calls (8 torch.cuda.Event) or None."""
        if events is None:
            check(lib().sg_batch_set_events(self._h, None, 0), "sg_batch_set_events")
            return
        for e in events:
            if not e.cuda_event:
                e.record()
        torch.cuda.synchronize()
        arr = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
        check(lib().sg_batch_set_events(self._h, arr, len(events)), "sg_batch_set_events")

    def solve(self, f, u0, v0, U, stream=None):
        """Batched forward: lists of device tensors (one per problem)."""
        check(lib().sg_batch_solve(self._h, self._ptrs(f, False, "f"), self._ptrs(u0, True, "u0"),
                                   self._ptrs(v0, True, "v0"), self._ptrs(U, False, "U"),
                                   _stream(stream)), "sg_batch_solve")

    def adjoint(self, g, df=None, du0=None, dv0=None, stream=None):
        """Batched adjoint; df / du0 / dv0 lists (or entries) may be None."""
        check(lib().sg_batch_adjoint(self._h, self._ptrs(g, False, "g"),
                                     self._ptrs(df, False, "df", True),
                                     self._ptrs(du0, True, "du0", True),
                                     self._ptrs(dv0, True, "dv0", True), _stream(stream)),
              "sg_batch_adjoint")

    def capture(self, f, u0, v0, U, g=None, df=None, du0=None, dv0=None, stream=None):
        """Lists (one entry per problem) of device tensors, shapes as for
        SparseGridWave; g/df/du0/dv0 may be None (forward only)."""
        P = self._ptrs
        args = [P(f, False, "f"), P(u0, True, "u0"), P(v0, True, "v0"), P(U, False, "U"),
                P(g, False, "g"), P(df, False, "df", True), P(du0, True, "du0", True),
                P(dv0, True, "dv0", True)]
        self._keep = (f, u0, v0, U, g, df, du0, dv0)  # buffers referenced by the graph
        check(lib().sg_batch_capture(self._h, *args, _stream(stream)), "sg_batch_capture")

    def replay(self, stream=None):
        check(lib().sg_batch_launch(self._h, _stream(stream)), "sg_batch_launch")


class SGWaveFunction(torch.autograd.Function):
    """U = F(f, u0, v0); backward applies the hand-written adjoint F^T."""

    @staticmethod
    def forward(ctx, solver, f, u0, v0):
        ctx.solver = solver
        return solver.solve(f.contiguous(), u0.contiguous(), v0.contiguous())

    @staticmethod
    def backward(ctx, gU):
        df, du0, dv0 = ctx.solver.adjoint(gU.contiguous())
        return None, df, du0, dv0


def tuning_status():
    """Which shape classes this process looked up in the tuning cache."""
    from . import autotune
    return autotune.status()


def sgwave(solver, f, u0, v0):
    """Differentiable forward map (autograd through the adjoint)."""
    return SGWaveFunction.apply(solver, f, u0, v0)
