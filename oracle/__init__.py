"""CPU oracle for the GS cascadic multigrid Fiedler solver (ctypes wrapper of
``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke``
and by the benchmark's CPU-baseline leg.  The library under
``paper_1602_04386_amd`` never imports or links it, and the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID, E_NOT_SYMMETRIC, E_NOT_LAPLACIAN, E_ISOLATED, E_NOMEM, E_NOT_CONVERGED = (
    0, -1, -2, -3, -4, -5, -7)


# IEEE arithmetic everywhere: no fast-math, no contraction into fused
# multiply-adds (-std=c99 already implies -ffp-contract=off; stated anyway), so
# every build computes bitwise the same results.
_FLAGS = ["-std=c99", "-ffp-contract=off", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compiles oracle.c with gcc (portable, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", *_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def host_cpu() -> dict:
    """The host's CPU model and the threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


def build_native() -> str:
    """Compiles oracle.c with -O3 -march=native for the timing baseline.  The
    library's name carries a hash of this host's CPU model and flags, so a copy
    built on another machine is never loaded here."""
    import hashlib

    key = ""
    try:
        with open("/proc/cpuinfo") as f:
            key = "".join(l for l in f if l.startswith(("model name", "flags")))
    except OSError:
        pass
    tag = hashlib.sha256(key.encode()).hexdigest()[:12]
    path = os.path.join(_HERE, f"liboracle_native_{tag}.so")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=native", *_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def use_native():
    """Loads the -O3 -march=native build (built here if needed) in place of the
    portable one; must be called before the first use of the oracle."""
    global _LIB, _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _LIB = build_native()
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        L.or_pair_hash.restype = C.c_uint32
        L.or_pair_hash.argtypes = [C.c_int32, C.c_int32]
        L.or_level_seed.restype = C.c_uint32
        L.or_level_seed.argtypes = [C.c_uint64, C.c_int32]
        L.or_can_reach.restype = C.c_int32
        L.or_can_reach.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32]
        L.or_colour_priority.restype = C.c_uint32
        L.or_colour_priority.argtypes = [C.c_int32, C.c_uint32]
        L.or_input_to_adjacency.restype = C.c_int32
        L.or_input_to_adjacency.argtypes = [C.c_int32, C.c_int64, i32p, i32p, f64p, C.c_int32,
                                            i32p, i32p, f64p, C.POINTER(C.c_int64)]
        L.or_match.restype = C.c_int32
        L.or_match.argtypes = [C.c_int32, i32p, i32p, f64p, i32p]
        L.or_aggregate.restype = C.c_int32
        L.or_aggregate.argtypes = [C.c_int32, i32p, i32p, f64p, i32p, i32p]
        L.or_galerkin.restype = C.c_int32
        L.or_galerkin.argtypes = [C.c_int32, i32p, i32p, f64p, i32p, C.c_int32, i32p, i32p,
                                  f64p, C.POINTER(C.c_int64)]
        L.or_colour.restype = C.c_int32
        L.or_colour.argtypes = [C.c_int32, i32p, i32p, C.c_uint32, i32p]
        L.or_recolour.restype = C.c_int32
        L.or_recolour.argtypes = [C.c_int32, i32p, i32p, C.c_int32, i32p]
        L.or_hec_random.restype = C.c_int32
        L.or_hec_random.argtypes = [C.c_int32, i32p, i32p, f64p, i32p, i32p]
        L.or_randperm.restype = None
        L.or_randperm.argtypes = [C.c_int32, C.c_uint64, i32p]
        L.or_colour_two.restype = C.c_int32
        L.or_colour_two.argtypes = [C.c_int32, i32p, i32p, i32p]
        L.or_level_colouring.restype = C.c_int32
        L.or_level_colouring.argtypes = [C.c_int32, i32p, i32p, C.c_uint32, C.c_int32, i32p]
        L.or_sigma.restype = C.c_double
        L.or_sigma.argtypes = [C.c_int32, i32p, f64p]
        L.or_pi_apply.restype = None
        L.or_pi_apply.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_double, f64p, f64p]
        L.or_gs_sweep.restype = None
        L.or_gs_sweep.argtypes = [C.c_int32, i32p, i32p, f64p, i32p, C.c_int32, C.c_double,
                                  C.c_double, f64p]
        L.or_gs_sweep_lex.restype = None
        L.or_gs_sweep_lex.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_double, f64p]
        L.or_rq_export.restype = C.c_double
        L.or_rq_export.argtypes = [C.c_int32, i32p, i32p, f64p, f64p]
        L.or_project_normalise_export.restype = None
        L.or_project_normalise_export.argtypes = [C.c_int32, f64p]
        L.or_rq_residual.restype = None
        L.or_rq_residual.argtypes = [C.c_int32, i32p, i32p, f64p, f64p, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.or_random_start.restype = None
        L.or_random_start.argtypes = [C.c_int32, C.c_uint64, f64p]
        L.or_coarsest.restype = C.c_int32
        L.or_coarsest.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_double, C.c_uint64, C.c_int32,
                                  C.c_int32, C.c_double, f64p, C.POINTER(C.c_int32)]
        L.or_fix_sign.restype = None
        L.or_fix_sign.argtypes = [C.c_int32, f64p]
        L.or_hier_build.restype = C.c_void_p
        L.or_hier_build.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, C.c_int32, C.c_uint64,
                                    C.POINTER(C.c_int32)]
        L.or_hier_build_hec.restype = C.c_void_p
        L.or_hier_build_hec.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, C.c_int32,
                                        C.c_uint64, C.c_uint64, C.POINTER(C.c_int32)]
        L.or_hier_free.restype = None
        L.or_hier_free.argtypes = [C.c_void_p]
        L.or_hier_nlevels.restype = C.c_int32
        L.or_hier_nlevels.argtypes = [C.c_void_p]
        L.or_hier_level_info.restype = C.c_double
        L.or_hier_level_info.argtypes = [C.c_void_p, C.c_int32, i64p]
        L.or_hier_level_copy.restype = None
        L.or_hier_level_copy.argtypes = [C.c_void_p, C.c_int32, i32p, i32p, f64p, C.c_void_p,
                                         C.c_void_p]
        L.or_solve.restype = C.c_int32
        L.or_solve.argtypes = [C.c_void_p, C.c_void_p, f64p, f64p, i32p, C.c_int32,
                               C.POINTER(C.c_int32)]
        _lib = L
    return _lib


class SolveParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("tol_cos", C.c_double), ("tol_res", C.c_double),
                ("max_gs", C.c_int32), ("max_pi", C.c_int32), ("max_outer", C.c_int32),
                ("max_coarsest", C.c_int32), ("gs_lexicographic", C.c_int32),
                ("gs_unshifted", C.c_int32), ("omega", C.c_double),
                ("replay", C.POINTER(C.c_int32)), ("replay_len", C.c_int32),
                ("tol_coarse", C.c_double), ("coarse_mass", C.c_int32), ("gs_rhs_y", C.c_int32),
                ("lanczos_k", C.c_int32), ("early_exit", C.c_int32)]


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- single steps -------------------------------------------------------------

def input_to_adjacency(n, rowptr, col, val, is_adjacency):
    rowptr, col, val = _i32(rowptr), _i32(col), _f64(val)
    nnz = int(col.shape[0])
    orp = np.zeros(n + 1 if n >= 0 else 1, np.int32)
    ocol = np.zeros(max(nnz, 1), np.int32)
    ow = np.zeros(max(nnz, 1), np.float64)
    m = C.c_int64(0)
    if col.shape[0] == 0:
        col = np.zeros(1, np.int32)
        val = np.zeros(1, np.float64)
    st = lib().or_input_to_adjacency(n, nnz, rowptr, col, val, int(is_adjacency), orp, ocol, ow,
                                     C.byref(m))
    if st != OK:
        return st, None
    return st, (orp, ocol[:m.value].copy(), ow[:m.value].copy())


def match(n, rowptr, col, w):
    mate = np.zeros(n, np.int32)
    st = lib().or_match(n, _i32(rowptr), _i32(col), _f64(w), mate)
    assert st == OK
    return mate


def aggregate(n, rowptr, col, w, mate):
    q = np.zeros(n, np.int32)
    nc = lib().or_aggregate(n, _i32(rowptr), _i32(col), _f64(w), _i32(mate), q)
    assert nc >= 0, nc
    return q, nc


def galerkin(n, rowptr, col, w, q, nc):
    m = int(col.shape[0])
    orp = np.zeros(nc + 1, np.int32)
    ocol = np.zeros(max(m, 1), np.int32)
    ow = np.zeros(max(m, 1), np.float64)
    mc = C.c_int64(0)
    st = lib().or_galerkin(n, _i32(rowptr), _i32(col), _f64(w), _i32(q), nc, orp, ocol, ow,
                           C.byref(mc))
    assert st == OK
    return orp, ocol[:mc.value].copy(), ow[:mc.value].copy()


def colour(n, rowptr, col, level_seed):
    c = np.zeros(n, np.int32)
    k = lib().or_colour(n, _i32(rowptr), _i32(col), level_seed, c)
    assert k >= 0
    return c, k


def recolour(n, rowptr, col, colour_in, ncol):
    """One iterated-greedy pass over a colouring; returns (colour, count)."""
    c = np.array(colour_in, dtype=np.int32, copy=True)
    k = lib().or_recolour(n, _i32(rowptr), _i32(col), ncol, c)
    assert k >= 0
    return c, k


def hec_random(n, rowptr, col, w, perm):
    """Algorithm 1 (randomised heavy edge coarsening) in the visiting order
    perm; returns (q, number of aggregates)."""
    q = np.zeros(n, np.int32)
    c = lib().or_hec_random(n, _i32(rowptr), _i32(col), _f64(w), _i32(perm), q)
    assert c >= 0
    return q, c


def randperm(n, seed):
    p = np.zeros(n, np.int32)
    lib().or_randperm(n, seed, p)
    return p


def colour_two(n, rowptr, col):
    """Two-colouring of a bipartite graph (each component's smallest vertex
    colour 0); returns (colour, count) with count 0 when the graph has an odd
    cycle."""
    c = np.zeros(n, np.int32)
    k = lib().or_colour_two(n, _i32(rowptr), _i32(col), c)
    assert k >= 0
    return c, k


def level_colouring(n, rowptr, col, level_seed, finest=True):
    """The smoother's colouring of a level: two colours when the finest level
    is bipartite, else first-fit in priority order plus one iterated-greedy
    pass."""
    c = np.zeros(n, np.int32)
    k = lib().or_level_colouring(n, _i32(rowptr), _i32(col), level_seed, int(finest), c)
    assert k >= 0
    return c, k


def level_seed(colour_seed, level):
    return lib().or_level_seed(colour_seed, level)


def can_reach(res, res_prev, tol, left):
    """or_can_reach: the finest rounds' early-exit test."""
    return bool(lib().or_can_reach(res, res_prev, tol, left))


def pair_hash(a, b):
    return lib().or_pair_hash(a, b)


def colour_priority(v, seed):
    return lib().or_colour_priority(v, seed)


def sigma(n, rowptr, w):
    return lib().or_sigma(n, _i32(rowptr), _f64(w))


def pi_apply(n, rowptr, col, w, sig, x):
    y = np.zeros(n)
    lib().or_pi_apply(n, _i32(rowptr), _i32(col), _f64(w), sig, _f64(x), y)
    return y


def gs_sweep(n, rowptr, col, w, colours, ncolours, x, rho=0.0, omega=1.0):
    x = _f64(x).copy()
    lib().or_gs_sweep(n, _i32(rowptr), _i32(col), _f64(w), _i32(colours), ncolours, rho, omega,
                      x)
    return x


def gs_sweep_lex(n, rowptr, col, w, x, rho=0.0):
    x = _f64(x).copy()
    lib().or_gs_sweep_lex(n, _i32(rowptr), _i32(col), _f64(w), rho, x)
    return x


def rayleigh(n, rowptr, col, w, x):
    return lib().or_rq_export(n, _i32(rowptr), _i32(col), _f64(w), _f64(x))


def project_normalise(x):
    x = _f64(x).copy()
    lib().or_project_normalise_export(x.shape[0], x)
    return x


def rq_residual(n, rowptr, col, w, x):
    rho, res = C.c_double(0), C.c_double(0)
    lib().or_rq_residual(n, _i32(rowptr), _i32(col), _f64(w), _f64(x), C.byref(rho),
                         C.byref(res))
    return rho.value, res.value


def random_start(n, seed):
    x = np.zeros(n)
    lib().or_random_start(n, seed, x)
    return x


def coarsest(n, rowptr, col, w, sig, seed, max_it=100000, replay_it=-1, tol=1e-13):
    x = np.zeros(n)
    conv = C.c_int32(0)
    it = lib().or_coarsest(n, _i32(rowptr), _i32(col), _f64(w), sig, seed, max_it, replay_it, tol,
                           x, C.byref(conv))
    return x, it, bool(conv.value)


# --- hierarchy and solve -----------------------------------------------------

@dataclass
class Level:
    n: int
    m: int
    rowptr: np.ndarray
    col: np.ndarray
    w: np.ndarray
    q: np.ndarray | None
    colour: np.ndarray | None
    ncolours: int
    sigma: float


@dataclass
class SolveResult:
    status: int
    x: np.ndarray
    lam: float
    residual: float
    final_cos: float
    counts: list = field(default_factory=list)


class Hierarchy:
    """Hierarchy built by the oracle (Algorithm 3, Step 1)."""

    def __init__(self, n, rowptr, col, w, n_coarse=25, max_levels=64, colour_seed=0,
                 hec_seed=0):
        """hec_seed != 0: the paper's randomised heavy edge coarsening
        (Algorithm 1 in random visiting orders) instead of the deterministic
        matching; an oracle-only mode."""
        st = C.c_int32(0)
        self._rp, self._col, self._w = _i32(rowptr), _i32(col), _f64(w)
        self._h = lib().or_hier_build_hec(n, self._rp, self._col, self._w, n_coarse, max_levels,
                                          colour_seed, hec_seed, C.byref(st))
        if not self._h:
            raise RuntimeError(f"oracle hierarchy build failed: {st.value}")
        self.nlevels = lib().or_hier_nlevels(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_hier_free(h)
            self._h = None

    def level(self, l) -> Level:
        info = np.zeros(3, np.int64)
        sig = lib().or_hier_level_info(self._h, l, info)
        n, m, k = (int(v) for v in info)
        rp = np.zeros(n + 1, np.int32)
        col = np.zeros(max(m, 1), np.int32)
        w = np.zeros(max(m, 1))
        last = l == self.nlevels - 1
        q = None if last else np.zeros(n, np.int32)
        c = None if last else np.zeros(n, np.int32)
        lib().or_hier_level_copy(self._h, l, rp, col, w,
                                 None if q is None else q.ctypes.data,
                                 None if c is None else c.ctypes.data)
        return Level(n, m, rp, col[:m], w[:m], q, c, k, sig)

    def solve(self, seed=1, tol_cos=1e-6, tol_res=0.0, max_gs=100, max_pi=100, max_outer=50,
              max_coarsest=100000, lexicographic=False, unshifted=False, omega=1.0,
              replay=None, tol_coarse=1e-13, coarse_mass=False, rhs_y=False,
              lanczos_k=0, early_exit=False) -> SolveResult:
        """Algorithm 3, Steps 2-3, then the finest Rayleigh quotient.  Variants
        (oracle-only, for comparison): lexicographic (Algorithm 2's row
        order), unshifted (the sweep on L x = 0), rhs_y (the sweep on L x = y),
        coarse_mass (coarse problems L_c y = lambda M_c y), lanczos_k (k
        Lanczos steps in place of each smoothing phase).  early_exit: the
        finest rounds end once the residual cannot reach tol_res within the
        rounds left at its last reduction factor (or_can_reach)."""
        n0 = self.level(0).n if self.nlevels else 0
        x = np.zeros(n0)
        scal = np.zeros(3)
        cap = 2 * 64 + 2 * max(max_outer, 0) + 8 + (len(replay) if replay is not None else 0)
        counts = np.zeros(cap, np.int32)
        clen = C.c_int32(0)
        P = SolveParams(seed, tol_cos, tol_res, max_gs, max_pi, max_outer, max_coarsest,
                        1 if lexicographic else 0, 1 if unshifted else 0, omega, None, 0,
                        tol_coarse, int(coarse_mass), int(rhs_y), int(lanczos_k), int(early_exit))
        keep = None
        if replay is not None:
            keep = (C.c_int32 * len(replay))(*[int(v) for v in replay])
            P.replay = C.cast(keep, C.POINTER(C.c_int32))
            P.replay_len = len(replay)
        st = lib().or_solve(self._h, C.byref(P), x, scal, counts, cap, C.byref(clen))
        return SolveResult(st, x, float(scal[0]), float(scal[1]), float(scal[2]),
                           [int(v) for v in counts[:clen.value]])


def solve_graph(g, n_coarse=25, colour_seed=0, **kw):
    """Builds the hierarchy of adjacency CSR ``g`` and solves."""
    h = Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=n_coarse, colour_seed=colour_seed)
    return h, h.solve(**kw)


def spectral_partition(g, parts, cut="median", vector=None, n_coarse=25, **solve_kw):
    """Recursive spectral bisection, the oracle's counterpart of the library's
    partitioning: log2(parts) rounds; in each, part p's induced subgraph
    (vertices of p with an edge inside p, in index order) is solved and cut in
    two -- median: the nsub // 2 smallest (value, index) pairs go to 2p;
    sign: phi_2 < 0 goes to 2p -- and the vertices of p without an edge inside
    p join the smaller half (2p on a tie).  vector(sub) returns the Fiedler
    vector of a subgraph (sub has n, rowptr, col, w); by default the oracle's
    own solve.  Returns (labels, number of vertices that were isolated in
    their part at some round)."""
    class Sub:
        pass

    if vector is None:
        def vector(sub):
            return Hierarchy(sub.n, sub.rowptr, sub.col, sub.w, n_coarse=n_coarse).solve(
                **solve_kw).x

    n = g.n
    rp = np.asarray(g.rowptr, np.int64)
    col = np.asarray(g.col, np.int64)
    w = np.asarray(g.w, np.float64)
    rows = np.repeat(np.arange(n), np.diff(rp))
    levels = int(np.log2(parts))
    part = np.zeros(n, np.int64)
    n_iso = 0
    for d in range(levels):
        nxt = part.copy()
        for p in range(2 ** d):
            mask = part == p
            inside = mask[rows] & mask[col]
            deg = np.bincount(rows[inside], minlength=n)
            inn = mask & (deg > 0)
            iso = mask & (deg == 0)
            n_iso += int(iso.sum())
            orig = np.nonzero(inn)[0]
            nsub = len(orig)
            c0 = c1 = 0
            if nsub >= 2:
                newid = np.cumsum(inn) - inn
                sub = Sub()
                sub.n = nsub
                sub.rowptr = np.concatenate([[0], np.cumsum(deg[orig])]).astype(np.int32)
                sub.col = newid[col[inside]].astype(np.int32)
                sub.w = w[inside].copy()
                x = np.asarray(vector(sub), np.float64) + 0.0
                child = np.ones(nsub, np.int64)
                if cut == "median":
                    order = np.lexsort((np.arange(nsub), x))
                    child[order[:nsub // 2]] = 0
                else:
                    child[x < 0.0] = 0
                c0 = int((child == 0).sum())
                c1 = nsub - c0
                nxt[orig] = 2 * p + child
            nxt[iso] = 2 * p + (1 if c1 < c0 else 0)
        part = nxt
    return part.astype(np.int32), n_iso
