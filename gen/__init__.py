"""Seeded synthetic graph generators shared by the tests, the benchmark and the
oracle checks.

This module only *produces inputs*: weighted undirected graphs in CSR form.  It
holds none of the solver's arithmetic (no matching, colouring, coarsening,
smoothing or eigen-solving), so both the HIP library and the CPU oracle can be
fed from it without sharing any method code.

Every random draw comes from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used counter-style: draw ``i``
of stream ``seed`` is ``mix(seed + (i + 1) * GAMMA)``; a uniform double in
[0, 1) is ``(z >> 11) * 2**-53``.

The graph families stand in for the paper's test inputs (Section 4): its
University of Florida matrices are not available here, so uniform 2-D grids
(the paper's own synthetic family, Table 4.2), random geometric graphs and
Erdos-Renyi graphs with the shapes and weight distributions of the workloads
are generated instead.

All generators return adjacency CSR ``(n, rowptr int32[n+1], col int32[m],
w float64[m])``: no diagonal, columns strictly ascending in every row, values
symmetric bit for bit, weights > 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (variant 13 of Stafford's mixers)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+count-1`` of the SplitMix64 stream seeded ``seed``."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
    return _mix64(z)


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits."""
    z = splitmix64(seed, count, start)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def derive_seed(seed: int, index: int) -> int:
    """Per-item seed: first SplitMix64 draw of the stream seeded ``seed ^ index``."""
    return int(splitmix64(seed ^ index, 1)[0])


@dataclass
class Graph:
    """Adjacency CSR of a weighted undirected graph."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[m]
    w: np.ndarray  # float64[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def laplacian(self):
        """CSR of L = D - W with the weighted degree on the diagonal (Def. 2.1)."""
        return adjacency_to_laplacian(self.n, self.rowptr, self.col, self.w)

    def dense_laplacian(self) -> np.ndarray:
        A = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        A[rows, self.col] = self.w
        return np.diag(A.sum(axis=1)) - A


def _csr_from_undirected(n: int, a: np.ndarray, b: np.ndarray, w: np.ndarray, name=""):
    """Symmetric CSR from undirected edges a[k] < b[k] (no duplicates)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    vals = np.concatenate([w, w])
    order = np.argsort(rows * n + cols, kind="stable")
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    if rowptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, rowptr.astype(np.int32), cols.astype(np.int32), vals, name)


def path(n: int, weights: str = "unit", seed: int = 0) -> Graph:
    """Path graph 0-1-...-(n-1)."""
    a = np.arange(n - 1)
    w = np.ones(n - 1) if weights == "unit" else 0.5 + uniform01(seed, n - 1)
    return _csr_from_undirected(n, a, a + 1, w, f"path{n}")


def grid(rows: int, cols: int, weights: str = "unit", seed: int = 0, lo: float = 0.5,
         hi: float = 1.5) -> Graph:
    """rows x cols 5-point grid, vertex id = r*cols + c.

    Undirected edges are enumerated vertex by vertex in id order, the edge to the
    right neighbour before the edge to the neighbour below; with
    ``weights="uniform"`` edge k of that enumeration gets ``lo + (hi-lo)*u_k``.
    """
    r, c = np.divmod(np.arange(rows * cols, dtype=np.int64), cols)
    v = r * cols + c
    has_right = c + 1 < cols
    has_down = r + 1 < rows
    # interleave (right, down) per vertex to fix the enumeration order
    a = np.stack([v, v], axis=1).reshape(-1)
    b = np.stack([v + 1, v + cols], axis=1).reshape(-1)
    keep = np.stack([has_right, has_down], axis=1).reshape(-1)
    a, b = a[keep], b[keep]
    if weights == "unit":
        w = np.ones(a.shape[0])
    elif weights == "uniform":
        w = lo + (hi - lo) * uniform01(seed, a.shape[0])
    else:
        raise ValueError(weights)
    return _csr_from_undirected(rows * cols, a, b, w, f"grid{rows}x{cols}")


def grid_with_hub(rows: int, cols: int, stride: int, seed: int = 0) -> Graph:
    """rows x cols 5-point grid (weights U[0.5, 1.5] as ``grid(..., "uniform",
    seed)``) plus one hub vertex, id rows*cols, joined to every stride-th grid
    vertex with weight 1: a graph with one very long row among short ones."""
    g = grid(rows, cols, "uniform", seed=seed)
    n0 = rows * cols
    r = np.repeat(np.arange(n0, dtype=np.int64), np.diff(g.rowptr))
    upper = g.col > r
    a = np.concatenate([r[upper], np.arange(0, n0, stride, dtype=np.int64)])
    b = np.concatenate([g.col[upper].astype(np.int64),
                        np.full(len(range(0, n0, stride)), n0, dtype=np.int64)])
    w = np.concatenate([g.w[upper], np.ones(len(range(0, n0, stride)))])
    return _csr_from_undirected(n0 + 1, a, b, w, f"grid{rows}x{cols}hub{stride}")


def largest_component(g: Graph) -> Graph:
    """Largest connected component, vertices relabelled in their original order."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    A = csr_matrix((g.w, g.col, g.rowptr), shape=(g.n, g.n))
    ncomp, lab = connected_components(A, directed=False)
    if ncomp == 1:
        return g
    big = np.argmax(np.bincount(lab))
    keep = lab == big
    newid = np.cumsum(keep) - 1
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    sel = keep[rows]
    r2, c2, w2 = newid[rows[sel]], newid[g.col[sel]], g.w[sel]
    n2 = int(keep.sum())
    rowptr = np.zeros(n2 + 1, dtype=np.int64)
    np.add.at(rowptr, r2 + 1, 1)
    rowptr = np.cumsum(rowptr)
    # rows stay sorted and columns stay ascending because relabelling is monotone
    return Graph(n2, rowptr.astype(np.int32), c2.astype(np.int32), w2, g.name + "-lcc")


def rgg(n: int, seed: int, radius: float | None = None, lcc: bool = True,
        chunk: int = 1 << 20) -> Graph:
    """Random geometric graph in the unit square.

    Points are iid uniform (x = u_{2i}, y = u_{2i+1}); an edge joins points at
    distance d < r with weight exp(-d^2/r^2).  The default radius
    r = sqrt(8/(pi n)) gives mean degree about 8.  Vertices are numbered by
    grid cell of side >= r (cells row-major, ties by point index), then the
    largest connected component is kept.
    """
    r = math.sqrt(8.0 / (math.pi * n)) if radius is None else radius
    u = uniform01(seed, 2 * n)
    x, y = u[0::2], u[1::2]
    G = max(1, int(math.floor(1.0 / r)))
    cx = np.minimum((x * G).astype(np.int64), G - 1)
    cy = np.minimum((y * G).astype(np.int64), G - 1)
    cell = cy * G + cx
    order = np.argsort(cell, kind="stable")
    x, y, cell = x[order], y[order], cell[order]
    cx, cy = cx[order], cy[order]
    start = np.searchsorted(cell, np.arange(G * G + 1))
    r2 = r * r
    ea, eb, ew = [], [], []
    offsets = [(0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
    for p0 in range(0, n, chunk):
        p = np.arange(p0, min(n, p0 + chunk), dtype=np.int64)
        pcx, pcy = cx[p], cy[p]
        for dx, dy in offsets:
            qx, qy = pcx + dx, pcy + dy
            ok = (qx >= 0) & (qx < G) & (qy < G)
            pp = p[ok]
            tc = qy[ok] * G + qx[ok]
            lo = start[tc]
            hi = start[tc + 1]
            if dx == 0 and dy == 0:
                lo = np.maximum(lo, pp + 1)
            cnt = np.maximum(hi - lo, 0)
            tot = int(cnt.sum())
            if tot == 0:
                continue
            src = np.repeat(pp, cnt)
            base = np.repeat(lo - np.cumsum(cnt) + cnt, cnt)
            dst = base + np.arange(tot, dtype=np.int64)
            d2 = (x[src] - x[dst]) ** 2 + (y[src] - y[dst]) ** 2
            hit = d2 < r2
            src, dst, d2 = src[hit], dst[hit], d2[hit]
            ea.append(np.minimum(src, dst))
            eb.append(np.maximum(src, dst))
            ew.append(np.exp(-d2 / r2))
    a = np.concatenate(ea) if ea else np.zeros(0, np.int64)
    b = np.concatenate(eb) if eb else np.zeros(0, np.int64)
    w = np.concatenate(ew) if ew else np.zeros(0)
    g = _csr_from_undirected(n, a, b, w, f"rgg{n}")
    return largest_component(g) if lcc else g


def erdos_renyi(n: int, p: float, seed: int, lcc: bool = True, lo: float = 0.5,
                hi: float = 1.5) -> Graph:
    """G(n, p) by geometric skipping over the pairs i < j in row-major order
    (Batagelj & Brandes 2005); weights U[lo, hi]; largest component kept."""
    N = n * (n - 1) // 2
    logq = math.log1p(-p)
    picks = []
    pos = -1
    drawn = 0
    block = max(1024, int(p * N * 1.1) + 64)
    while True:
        u = uniform01(seed, block, start=drawn)
        drawn += block
        skips = np.floor(np.log1p(-u) / logq).astype(np.int64) + 1
        idx = pos + np.cumsum(skips)
        inside = idx < N
        picks.append(idx[inside])
        if not inside.all():
            break
        pos = int(idx[-1])
    lin = np.concatenate(picks)
    # row i of the strict upper triangle starts at off(i) = i*n - i*(i+1)/2
    ii = np.arange(n, dtype=np.int64)
    off = ii * n - ii * (ii + 1) // 2
    a = np.searchsorted(off, lin, side="right") - 1
    b = lin - off[a] + a + 1
    w = lo + (hi - lo) * uniform01(seed ^ 0x5EED, lin.shape[0])
    g = _csr_from_undirected(n, a, b, w, f"er{n}")
    return largest_component(g) if lcc else g


def random_connected(n: int, seed: int, extra: float = 1.5, dyadic: bool = False) -> Graph:
    """Small random connected graph: a random spanning tree plus ~extra*n random
    edges.  With ``dyadic`` the weights are multiples of 1/8 in [1/8, 2], so
    every sum of them is exact in binary floating point."""
    u = uniform01(seed, 4 * n + 8 * int(extra * n) + 16)
    k = 0
    edges = {}
    for v in range(1, n):
        parent = int(u[k] * v)
        k += 1
        edges[(parent, v)] = None
    tries = int(extra * n)
    for _ in range(tries):
        a = int(u[k] * n)
        b = int(u[k + 1] * n)
        k += 2
        if a != b:
            edges[(min(a, b), max(a, b))] = None
    pairs = sorted(edges)
    a = np.array([p[0] for p in pairs], dtype=np.int64)
    b = np.array([p[1] for p in pairs], dtype=np.int64)
    uw = uniform01(seed ^ 0xABCDEF, len(pairs))
    if dyadic:
        w = (1.0 + np.floor(uw * 16.0)) / 8.0
    else:
        w = 0.5 + uw
    return _csr_from_undirected(n, a, b, w, f"rand{n}")


def adjacency_to_laplacian(n, rowptr, col, w):
    """CSR of L = D - W (diagonal inserted in column order)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    deg = np.zeros(n)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    np.add.at(deg, rows, w)
    r2 = np.concatenate([rows, np.arange(n)])
    c2 = np.concatenate([np.asarray(col, np.int64), np.arange(n)])
    v2 = np.concatenate([-np.asarray(w), deg])
    order = np.argsort(r2 * n + c2, kind="stable")
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r2 + 1, 1)
    return (np.cumsum(rp).astype(np.int32), c2[order].astype(np.int32), v2[order])


# --- the benchmark workloads, as concrete seeded inputs -----------------------

def grid_32x24() -> Graph:
    """32 x 24 unit-weight grid, n = 768 (the small plain-FP64 workload)."""
    return grid(32, 24, "unit")


def grid_1024x1000(seed: int = 2) -> Graph:
    """1024 x 1000 grid with iid U[0.5, 1.5] weights, n = 1,024,000."""
    return grid(1024, 1000, "uniform", seed=seed)


def rgg_4m(seed: int = 3, n: int = 4_000_000) -> Graph:
    """Random geometric graph with 4M points, mean degree ~8, LCC."""
    return rgg(n, seed)


def batch_mix(count: int = 4096, seed: int = 4, nmin: int = 200, nmax: int = 50000):
    """Mixed batch: n log-uniform in [nmin, nmax]; a seeded coin picks a 4:3
    grid with U[0.5,1.5] weights or G(n, 6/(n-1)) (LCC) with U[0.5,1.5]."""
    out = []
    for g in range(count):
        s = derive_seed(seed, g)
        u = uniform01(s, 2)
        n = int(round(math.exp(math.log(nmin) + u[0] * (math.log(nmax) - math.log(nmin)))))
        if u[1] < 0.5:
            a = int(round(math.sqrt(4.0 * n / 3.0)))
            b = max(2, int(round(n / a)))
            out.append(grid(a, b, "uniform", seed=s ^ 0x77))
        else:
            out.append(erdos_renyi(n, 6.0 / (n - 1), seed=s ^ 0x99))
    return out


def serve_pool(count: int = 32, seed: int = 5, nmin: int = 1000, nmax: int = 2_000_000,
               progress=None):
    """Pool of request graphs: n log-uniform in [nmin, nmax]; a seeded coin
    picks a random geometric graph (probability 0.7, largest component) or a
    4:3 grid with U[0.5,1.5] weights.  Graph g depends on (seed, g) alone, so
    a pool is a prefix of any larger one.  progress(g), if given, is called
    before graph g is generated."""
    out = []
    for g in range(count):
        if progress is not None:
            progress(g)
        s = derive_seed(seed, g)
        u = uniform01(s, 2)
        n = int(round(math.exp(math.log(nmin) + u[0] * (math.log(nmax) - math.log(nmin)))))
        if u[1] < 0.7:
            out.append(rgg(n, s ^ 0x55))
        else:
            a = int(round(math.sqrt(4.0 * n / 3.0)))
            b = max(2, int(round(n / a)))
            out.append(grid(a, b, "uniform", seed=s ^ 0x33))
    return out


def poisson_arrivals(rate: float, duration: float, seed: int = 5) -> np.ndarray:
    """Arrival times in [0, duration) of a Poisson process of the given rate:
    exponential gaps -ln(1 - u) / rate from SplitMix64 uniforms."""
    count = int(rate * duration * 1.5) + 64
    u = uniform01(seed, count)
    t = np.cumsum(-np.log1p(-u) / rate)
    return t[t < duration]
