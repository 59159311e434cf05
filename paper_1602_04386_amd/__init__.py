"""Python binding of the MI355X Fiedler-vector library (``include/fiedler.h``).

Argument marshalling only: every step of the solver runs in the HIP library
``libfiedler.so``.  Importing this package fails loudly when the library is
missing; there is no fallback.  Device arrays may be passed as torch tensors
(torch is used for device memory and streams only).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfiedler.so")

FV_MAX_LEVELS = 64
FV_SCHEDULE_CAP = 1024

STATUS = {0: "OK", 1: "PENDING", -1: "E_INVALID", -2: "E_NOT_SYMMETRIC", -3: "E_NOT_LAPLACIAN",
          -4: "E_ISOLATED", -5: "E_NOMEM", -6: "E_BUDGET", -7: "E_NOT_CONVERGED",
          -8: "E_DEVICE", -9: "E_UNKNOWN_TICKET", -10: "E_BUSY", -11: "E_SCRATCH"}
OK, PENDING, E_INVALID, E_NOT_SYMMETRIC, E_NOT_LAPLACIAN, E_ISOLATED = 0, 1, -1, -2, -3, -4
E_NOMEM, E_BUDGET, E_NOT_CONVERGED, E_DEVICE, E_UNKNOWN_TICKET, E_BUSY = -5, -6, -7, -8, -9, -10
E_SCRATCH = -11
NOALLOC_SCRATCH_BYTES = 32 << 20  # FV_NOALLOC_SCRATCH_BYTES
PREC = {"fp64": 0, "fp32": 1, "fp32_mixed": 1}


class FiedlerError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


class fv_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("is_adjacency", C.c_int32),
                ("on_device", C.c_int32)]


class fv_hier_opts(C.Structure):
    _fields_ = [("n_coarse", C.c_int32), ("max_levels", C.c_int32), ("colour_seed", C.c_uint64),
                ("ell", C.c_int32)]


class fv_solve_opts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("seed", C.c_uint64), ("tol_cos", C.c_double),
                ("tol_res", C.c_double), ("omega", C.c_double), ("max_gs", C.c_int32),
                ("max_pi", C.c_int32), ("max_outer", C.c_int32), ("max_coarsest", C.c_int32),
                ("replay", C.POINTER(C.c_int32)), ("replay_len", C.c_int32),
                ("stream", C.c_void_p), ("tol_coarse", C.c_double), ("time_finest", C.c_int32),
                ("early_exit", C.c_int32)]


class fv_solve_stats(C.Structure):
    _fields_ = [("levels", C.c_int32), ("n", C.c_int32 * FV_MAX_LEVELS),
                ("nnz", C.c_int64 * FV_MAX_LEVELS), ("colours", C.c_int32 * FV_MAX_LEVELS),
                ("schedule_len", C.c_int32), ("schedule", C.c_int32 * FV_SCHEDULE_CAP),
                ("lambda_", C.c_double), ("residual", C.c_double), ("final_cos", C.c_double),
                ("t_solve_ms", C.c_double), ("alg_bytes", C.c_int64),
                ("n_finest_gs", C.c_int32), ("t_finest_gs_ms", C.c_double),
                ("finest_gs_bytes", C.c_int64)]


class fv_batch_opts(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("graph", C.c_int32), ("lds_bytes", C.c_int64),
                ("lds_bytes_used", C.c_int64), ("grid", C.c_int32), ("tuned", C.c_int32),
                ("replayed", C.c_int32), ("launch_ms", C.c_double)]


class fv_partition_opts(C.Structure):
    _fields_ = [("parts", C.c_int32), ("cut", C.c_int32)]


class fv_partition_stats(C.Structure):
    _fields_ = [("parts", C.c_int32), ("part_size_min", C.c_int32), ("part_size_max", C.c_int32),
                ("solves", C.c_int32), ("not_converged", C.c_int32), ("cut_weight", C.c_double),
                ("total_weight", C.c_double), ("t_ms", C.c_double)]


class fv_server_opts(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("queue_capacity", C.c_int32),
                ("hbm_budget_bytes", C.c_size_t), ("cache_hierarchies", C.c_int32),
                ("hier", fv_hier_opts), ("solve", fv_solve_opts), ("workers", C.c_int32)]


class fv_request(C.Structure):
    _fields_ = [("graph_id", C.c_uint64), ("graph", C.POINTER(fv_csr)), ("x_out", C.c_void_p)]


class fv_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("lambda_", C.c_double), ("residual", C.c_double),
                ("queue_ms", C.c_double), ("latency_ms", C.c_double), ("cache_hit", C.c_int32),
                ("alg_bytes", C.c_int64)]


EXPORTS = ["fv_hier_opts_default", "fv_solve_opts_default", "fv_context_create",
           "fv_context_destroy", "fv_build_hierarchy", "fv_build_hierarchies", "fv_hierarchy_info", "fv_hierarchy_bytes",
           "fv_hierarchy_ell_width",
           "fv_hierarchy_export_level", "fv_free_hierarchy", "fv_fiedler_solve",
           "fv_fiedler_solve_noalloc", "fv_fiedler_solve_batch", "fv_fiedler_solve_batch_ex",
           "fv_batch_opts_default", "fv_spectral_partition", "fv_server_create", "fv_submit", "fv_poll",
           "fv_server_destroy", "fv_status_str"]

_lib = None


def lib() -> C.CDLL:
    """Loads libfiedler.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1602_04386_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.fv_hier_opts_default.argtypes = [C.POINTER(fv_hier_opts)]
        L.fv_hier_opts_default.restype = None
        L.fv_solve_opts_default.argtypes = [C.POINTER(fv_solve_opts)]
        L.fv_solve_opts_default.restype = None
        L.fv_context_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(vp)]
        L.fv_context_create.restype = C.c_int
        L.fv_context_destroy.argtypes = [vp]
        L.fv_context_destroy.restype = None
        L.fv_build_hierarchy.argtypes = [vp, C.POINTER(fv_csr), C.POINTER(fv_hier_opts),
                                         C.POINTER(vp)]
        L.fv_build_hierarchy.restype = C.c_int
        L.fv_build_hierarchies.argtypes = [vp, C.c_int32, C.POINTER(C.POINTER(fv_csr)),
                                           C.POINTER(fv_hier_opts), C.c_int32, C.POINTER(vp),
                                           C.POINTER(C.c_int)]
        L.fv_build_hierarchies.restype = C.c_int
        L.fv_hierarchy_info.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fv_hierarchy_info.restype = C.c_int
        L.fv_hierarchy_bytes.argtypes = [vp, C.POINTER(C.c_int64)]
        L.fv_hierarchy_bytes.restype = C.c_int
        L.fv_hierarchy_export_level.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp]
        L.fv_hierarchy_export_level.restype = C.c_int
        L.fv_free_hierarchy.argtypes = [vp]
        L.fv_free_hierarchy.restype = None
        L.fv_fiedler_solve.argtypes = [vp, vp, C.POINTER(fv_solve_opts), vp, C.c_int32,
                                       C.POINTER(C.c_double), C.POINTER(fv_solve_stats)]
        L.fv_fiedler_solve.restype = C.c_int
        L.fv_fiedler_solve_noalloc.argtypes = L.fv_fiedler_solve.argtypes
        L.fv_fiedler_solve_noalloc.restype = C.c_int
        L.fv_fiedler_solve_batch.argtypes = [vp, C.c_int32, vp, C.POINTER(fv_solve_opts), vp,
                                             C.c_int32, vp, vp, vp]
        L.fv_fiedler_solve_batch.restype = C.c_int
        L.fv_fiedler_solve_batch_ex.argtypes = [vp, C.c_int32, vp, C.POINTER(fv_solve_opts),
                                                C.POINTER(fv_batch_opts), vp, C.c_int32, vp, vp,
                                                vp]
        L.fv_fiedler_solve_batch_ex.restype = C.c_int
        L.fv_spectral_partition.argtypes = [vp, C.POINTER(fv_csr), C.POINTER(fv_hier_opts),
                                            C.POINTER(fv_solve_opts),
                                            C.POINTER(fv_partition_opts), vp, C.c_int32,
                                            C.POINTER(fv_partition_stats)]
        L.fv_spectral_partition.restype = C.c_int
        L.fv_batch_opts_default.argtypes = [C.POINTER(fv_batch_opts)]
        L.fv_batch_opts_default.restype = None
        L.fv_server_create.argtypes = [vp, C.POINTER(fv_server_opts), C.POINTER(vp)]
        L.fv_server_create.restype = C.c_int
        L.fv_submit.argtypes = [vp, C.POINTER(fv_request), C.POINTER(C.c_uint64)]
        L.fv_submit.restype = C.c_int
        L.fv_poll.argtypes = [vp, C.c_uint64, C.POINTER(fv_result)]
        L.fv_poll.restype = C.c_int
        L.fv_server_destroy.argtypes = [vp]
        L.fv_server_destroy.restype = None
        L.fv_status_str.argtypes = [C.c_int]
        L.fv_status_str.restype = C.c_char_p
        _lib = L
    return _lib


def status_str(st: int) -> str:
    return lib().fv_status_str(st).decode()


def _check(st: int, what: str):
    if st != OK:
        raise FiedlerError(st, what)


def _ptr(a):
    """(pointer, on_device, keepalive) of a numpy array or a torch tensor."""
    if hasattr(a, "data_ptr"):  # torch tensor
        return a.data_ptr(), int(a.is_cuda), a
    a = np.ascontiguousarray(a)
    return a.ctypes.data, 0, a


# --- context and hierarchy ------------------------------------------------------

_live_contexts: "weakref.WeakSet[Context]" = weakref.WeakSet()


@atexit.register
def _close_all_contexts():
    # Runs before the interpreter tears objects down in arbitrary order and
    # before the HIP runtime's own exit handlers: a context (and the
    # hierarchies and servers it owns) left open by the program is released
    # while the runtime still works.
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """A device context (one per thread)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().fv_context_create(device, hbm_budget_bytes, C.byref(h)), "fv_context_create")
        self._h = h
        self._children = weakref.WeakSet()  # hierarchies and servers of this context
        _live_contexts.add(self)

    @property
    def handle(self):
        if not self._h:
            raise FiedlerError(E_INVALID, "context is closed")
        return self._h

    def close(self):
        """Frees the context's servers and hierarchies, then the context."""
        if self._h:
            for child in sorted(self._children, key=lambda c: not isinstance(c, Server)):
                child.close()
            lib().fv_context_destroy(self._h)
            self._h = None

    def __del__(self):
        if sys.is_finalizing():
            return  # _close_all_contexts has run; never call HIP this late
        try:
            self.close()
        except Exception:
            pass


@dataclass
class LevelExport:
    n: int
    m: int
    rowptr: np.ndarray
    col: np.ndarray
    w: np.ndarray
    q: np.ndarray | None
    colour: np.ndarray | None
    ncolours: int
    sigma: float


class Hierarchy:
    def __init__(self, ctx: Context, handle: C.c_void_p):
        self.ctx = ctx
        self._h = handle
        ctx._children.add(self)
        self.levels, self.n, self.nnz, self.colours, self.sigma = self._info()

    def _info(self):
        lev = C.c_int32()
        n = (C.c_int32 * FV_MAX_LEVELS)()
        nnz = (C.c_int64 * FV_MAX_LEVELS)()
        col = (C.c_int32 * FV_MAX_LEVELS)()
        sig = (C.c_double * FV_MAX_LEVELS)()
        _check(lib().fv_hierarchy_info(self._h, C.addressof(lev), C.addressof(n),
                                       C.addressof(nnz), C.addressof(col), C.addressof(sig)),
               "fv_hierarchy_info")
        L = lev.value
        return L, list(n[:L]), list(nnz[:L]), list(col[:L]), list(sig[:L])

    def device_bytes(self) -> int:
        """fv_hierarchy_bytes: device memory the hierarchy holds."""
        b = C.c_int64()
        _check(lib().fv_hierarchy_bytes(self._h, C.byref(b)), "fv_hierarchy_bytes")
        return b.value

    def ell_width(self, level: int, colour: int = 0) -> int:
        """fv_hierarchy_ell_width: slots per row of the ELL block of a colour of
        a level (0: swept from CSR)."""
        w = C.c_int32()
        _check(lib().fv_hierarchy_ell_width(self._h, int(level), int(colour), C.byref(w)),
               "fv_hierarchy_ell_width")
        return w.value

    def export_level(self, level: int) -> LevelExport:
        n, m = self.n[level], self.nnz[level]
        rp = np.zeros(n + 1, np.int32)
        col = np.zeros(max(m, 1), np.int32)
        w = np.zeros(max(m, 1))
        last = level == self.levels - 1
        q = None if last else np.zeros(n, np.int32)
        c = None if last else np.zeros(n, np.int32)
        _check(lib().fv_hierarchy_export_level(self._h, level, rp.ctypes.data, col.ctypes.data,
                                               w.ctypes.data,
                                               None if q is None else q.ctypes.data,
                                               None if c is None else c.ctypes.data),
               "fv_hierarchy_export_level")
        return LevelExport(n, m, rp, col[:m], w[:m], q, c, self.colours[level], self.sigma[level])

    def free(self):
        if self._h:
            lib().fv_free_hierarchy(self._h)
            self._h = None

    close = free

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def _make_csr(n, rowptr, col, val, is_adjacency):
    rp, d0, k0 = _ptr(np.asarray(rowptr, np.int32) if not hasattr(rowptr, "data_ptr") else rowptr)
    cp, d1, k1 = _ptr(np.asarray(col, np.int32) if not hasattr(col, "data_ptr") else col)
    vp, d2, k2 = _ptr(np.asarray(val, np.float64) if not hasattr(val, "data_ptr") else val)
    if not (d0 == d1 == d2):
        raise ValueError("row_ptr, col and val must all be host arrays or all device tensors")
    nnz = int(col.shape[0]) if hasattr(col, "shape") else len(col)
    csr = fv_csr(int(n), nnz, rp, cp, vp, 1 if is_adjacency else 0, d0)
    return csr, (k0, k1, k2)


def build_hierarchy(ctx: Context, n: int, rowptr, col, val, is_adjacency: bool = True,
                    n_coarse: int = 25, max_levels: int = FV_MAX_LEVELS,
                    colour_seed: int = 0, ell: bool = True) -> Hierarchy:
    """fv_build_hierarchy: setup phase (Algorithm 3, Step 1) on the device.
    ell=False keeps every level in CSR only (fv_hier_opts.ell = -1)."""
    csr, keep = _make_csr(n, rowptr, col, val, is_adjacency)
    opts = fv_hier_opts(n_coarse, max_levels, colour_seed, 0 if ell else -1)
    h = C.c_void_p()
    _check(lib().fv_build_hierarchy(ctx.handle, C.byref(csr), C.byref(opts), C.byref(h)),
           "fv_build_hierarchy")
    del keep
    return Hierarchy(ctx, h)


def build_hierarchy_graph(ctx: Context, g, **kw) -> Hierarchy:
    return build_hierarchy(ctx, g.n, g.rowptr, g.col, g.w, True, **kw)


def build_hierarchies(ctx: Context, graphs, threads: int = 0, n_coarse: int = 25,
                      max_levels: int = FV_MAX_LEVELS, colour_seed: int = 0, ell: bool = True):
    """fv_build_hierarchies: the setup phase for many adjacency graphs (objects
    with n, rowptr, col, w) on concurrent host threads and streams.  Returns
    (hierarchies, statuses): a Hierarchy or None per graph, and its status."""
    count = len(graphs)
    csrs, keep = [], []
    for g in graphs:
        c, k = _make_csr(g.n, g.rowptr, g.col, g.w, True)
        csrs.append(c)
        keep.append(k)
    ptrs = (C.POINTER(fv_csr) * max(count, 1))(*[C.pointer(c) for c in csrs])
    out = (C.c_void_p * max(count, 1))()
    st = (C.c_int * max(count, 1))()
    opts = fv_hier_opts(n_coarse, max_levels, colour_seed, 0 if ell else -1)
    lib().fv_build_hierarchies(ctx.handle, count, ptrs, C.byref(opts), int(threads), out, st)
    del keep
    hs = [Hierarchy(ctx, C.c_void_p(out[i])) if out[i] else None for i in range(count)]
    return hs, [int(st[i]) for i in range(count)]


# --- solve ----------------------------------------------------------------------

@dataclass
class SolveResult:
    status: int
    x: object
    lam: float
    residual: float
    final_cos: float
    schedule: list = field(default_factory=list)
    t_solve_ms: float = 0.0
    alg_bytes: int = 0
    levels: int = 0
    n: list = field(default_factory=list)
    nnz: list = field(default_factory=list)
    colours: list = field(default_factory=list)
    n_finest_gs: int = 0
    t_finest_gs_ms: float = 0.0
    finest_gs_bytes: int = 0


def solve_opts(prec="fp64", seed=1, tol_cos=1e-6, tol_res=0.0, omega=1.0, max_gs=100,
               max_pi=100, max_outer=50, max_coarsest=100000, replay=None, stream=None,
               tol_coarse=1e-13, time_finest=False, early_exit=False):
    o = fv_solve_opts()
    lib().fv_solve_opts_default(C.byref(o))
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.seed, o.tol_cos, o.tol_res, o.omega = seed, tol_cos, tol_res, omega
    o.max_gs, o.max_pi, o.max_outer, o.max_coarsest = max_gs, max_pi, max_outer, max_coarsest
    o.tol_coarse = tol_coarse
    o.time_finest = 1 if time_finest else 0
    o.early_exit = 1 if early_exit else 0
    keep = None
    if replay is not None:
        keep = (C.c_int32 * len(replay))(*[int(v) for v in replay])
        o.replay = C.cast(keep, C.POINTER(C.c_int32))
        o.replay_len = len(replay)
    if stream is not None:
        o.stream = C.c_void_p(stream)
    return o, keep


def _stats_to_result(st, x, lam, S: fv_solve_stats) -> SolveResult:
    L = S.levels
    return SolveResult(st, x, lam, S.residual, S.final_cos, list(S.schedule[:S.schedule_len]),
                       S.t_solve_ms, S.alg_bytes, L, list(S.n[:L]), list(S.nnz[:L]),
                       list(S.colours[:L]), S.n_finest_gs, S.t_finest_gs_ms,
                       S.finest_gs_bytes)


def fiedler_solve(ctx: Context, h: Hierarchy, x_out=None, **kw) -> SolveResult:
    """fv_fiedler_solve.  x_out: optional device tensor of n float64; otherwise
    a host numpy array is returned."""
    return _solve(lib().fv_fiedler_solve, "fv_fiedler_solve", ctx, h, x_out, **kw)


def fiedler_solve_noalloc(ctx: Context, h: Hierarchy, x_out=None, **kw) -> SolveResult:
    """fv_fiedler_solve_noalloc: the same solve on the library's fixed device
    scratch, allocating nothing.  Raises FiedlerError(E_SCRATCH) when the
    hierarchy needs more than NOALLOC_SCRATCH_BYTES."""
    return _solve(lib().fv_fiedler_solve_noalloc, "fv_fiedler_solve_noalloc", ctx, h, x_out,
                  **kw)


def _solve(fn, name, ctx, h, x_out, **kw) -> SolveResult:
    o, keep = solve_opts(**kw)
    n0 = h.n[0]
    if x_out is None:
        x = np.zeros(n0)
        xp, on_dev = x.ctypes.data, 0
    else:
        x = x_out
        xp, on_dev = x_out.data_ptr(), 1
    lam = C.c_double()
    S = fv_solve_stats()
    st = fn(ctx.handle, h._h, C.byref(o), xp, on_dev, C.byref(lam), C.byref(S))
    del keep
    if st not in (OK, E_NOT_CONVERGED):
        raise FiedlerError(st, name)
    return _stats_to_result(st, x, lam.value, S)


def fiedler_solve_batch(ctx: Context, hs: list, x_out=None, batch=None, **kw) -> list:
    """fv_fiedler_solve_batch (fv_fiedler_solve_batch_ex when ``batch`` is a
    dict of launch options: autotune, graph, lds_bytes; the dict then receives
    the launch's lds_bytes_used, grid, tuned, replayed and launch_ms); returns
    one SolveResult per graph.  x_out: optional list of device arrays (n
    float64 each, data_ptr()); otherwise host numpy arrays are returned."""
    o, keep = solve_opts(**kw)
    bo = None
    if batch is not None:
        bo = fv_batch_opts()
        lib().fv_batch_opts_default(C.byref(bo))
        bo.autotune = int(batch.get("autotune", 0))
        bo.graph = int(batch.get("graph", 0))
        bo.lds_bytes = int(batch.get("lds_bytes", 0))
    count = len(hs)
    if x_out is None:
        xs = [np.zeros(h.n[0]) for h in hs]
        ptrs, on_dev = [x.ctypes.data for x in xs], 0
    else:
        if len(x_out) != count:
            raise ValueError("x_out needs one device array per hierarchy")
        xs = list(x_out)
        ptrs, on_dev = [x.data_ptr() for x in xs], 1
    hp = (C.c_void_p * count)(*[h._h.value for h in hs])
    xp = (C.c_void_p * count)(*ptrs)
    lam = (C.c_double * count)()
    stats = (fv_solve_stats * count)()
    ist = (C.c_int32 * count)()
    if bo is None:
        st = lib().fv_fiedler_solve_batch(ctx.handle, count, hp, C.byref(o), xp, on_dev, lam,
                                          stats, ist)
    else:
        st = lib().fv_fiedler_solve_batch_ex(ctx.handle, count, hp, C.byref(o), C.byref(bo), xp,
                                             on_dev, lam, stats, ist)
        batch.update(lds_bytes_used=bo.lds_bytes_used, grid=bo.grid, tuned=bool(bo.tuned),
                     replayed=bool(bo.replayed), launch_ms=bo.launch_ms)
    del keep
    _check(st, "fv_fiedler_solve_batch")
    return [_stats_to_result(ist[k], xs[k], lam[k], stats[k]) for k in range(count)]


# --- partitioning ---------------------------------------------------------------

def spectral_partition(ctx: Context, g, parts: int = 2, cut: str = "median", n_coarse: int = 25,
                       **solve_kw):
    """fv_spectral_partition on graph g (adjacency CSR with n, rowptr, col, w);
    returns (labels, stats dict)."""
    csr, keep = _make_csr(g.n, g.rowptr, g.col, g.w, True)
    ho = fv_hier_opts(n_coarse, FV_MAX_LEVELS, 0)
    o, keep2 = solve_opts(**solve_kw)
    po = fv_partition_opts(int(parts), {"median": 0, "sign": 1}[cut])
    out = np.zeros(g.n, np.int32)
    S = fv_partition_stats()
    _check(lib().fv_spectral_partition(ctx.handle, C.byref(csr), C.byref(ho), C.byref(o),
                                       C.byref(po), out.ctypes.data, 0, C.byref(S)),
           "fv_spectral_partition")
    del keep, keep2
    return out, {k: getattr(S, k) for k, _ in S._fields_}


# --- serving ----------------------------------------------------------------------

class Server:
    """fv_server_create / fv_submit / fv_poll / fv_server_destroy."""

    def __init__(self, ctx: Context, max_inflight=64, queue_capacity=4096, hbm_budget_bytes=0,
                 cache_hierarchies=True, n_coarse=25, workers=0, **solve_kw):
        so = fv_server_opts()
        so.max_inflight, so.queue_capacity = max_inflight, queue_capacity
        so.workers = workers
        so.hbm_budget_bytes, so.cache_hierarchies = hbm_budget_bytes, int(cache_hierarchies)
        so.hier = fv_hier_opts(n_coarse, FV_MAX_LEVELS, 0)
        o, keep = solve_opts(**solve_kw)
        if keep is not None:
            raise ValueError("replay is not supported by the server")
        so.solve = o
        h = C.c_void_p()
        _check(lib().fv_server_create(ctx.handle, C.byref(so), C.byref(h)), "fv_server_create")
        self._h = h
        self.ctx = ctx
        self._live = {}
        ctx._children.add(self)

    def submit(self, graph_id: int, g) -> int:
        """Queues a Fiedler request for graph ``g`` (adjacency CSR with fields n,
        rowptr, col, w) under ``graph_id``; the library reads ``g`` only when
        that id is not cached."""
        x = np.zeros(g.n)
        csr, keep = _make_csr(g.n, g.rowptr, g.col, g.w, True)
        csr_p = C.pointer(csr)
        req = fv_request(graph_id, csr_p, x.ctypes.data)
        t = C.c_uint64()
        _check(lib().fv_submit(self._h, C.byref(req), C.byref(t)), "fv_submit")
        self._live[t.value] = (x, keep, csr_p)
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (fv_result fields dict, x)."""
        r = fv_result()
        st = lib().fv_poll(self._h, ticket, C.byref(r))
        if st == PENDING:
            return None
        _check(st, "fv_poll")
        x, _, _ = self._live.pop(ticket)
        return ({"status": r.status, "lambda": r.lambda_, "residual": r.residual,
                 "queue_ms": r.queue_ms, "latency_ms": r.latency_ms,
                 "cache_hit": bool(r.cache_hit), "alg_bytes": r.alg_bytes}, x)

    def close(self):
        if self._h:
            lib().fv_server_destroy(self._h)
            self._h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
