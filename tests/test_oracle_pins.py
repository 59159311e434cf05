"""Pins of the CPU oracle against what the paper and the mathematics fix,
independently of the oracle's own code:

* closed forms: path and grid Laplacian spectra (lambda_2 = 2 - 2cos(pi/n) and
  2 - 2cos(pi/max(m,k)) for unit weights; the path Fiedler vector is
  cos(pi(i + 1/2)/n));
* dense brute force: numpy eigh on graphs of <= 64 vertices, the Galerkin
  product I L I^T formed densely, the Gauss-Seidel sweep written as a matrix
  splitting and solved with numpy, the power step as a dense product;
* independent algorithms: the locally dominant pointer-round matching and the
  Jones-Plassmann colouring simulated in Python must reproduce the oracle's
  sequential greedy matching and first-fit colouring;
* invariants: symmetry, zero row sums, connectivity, halving of levels, the
  eigenvector as a fixed point of the shifted sweep, Courant-Fischer against
  scipy's eigsh on a 30k-vertex grid.
"""
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import gen


def fmix32(h):
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    h ^= h >> 16
    return h


def pair_hash(a, b):
    return fmix32(fmix32(a) ^ b)


def dense_W(n, rp, col, w):
    A = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[rows, col] = w
    return A


def dense_L(n, rp, col, w):
    A = dense_W(n, rp, col, w)
    return np.diag(A.sum(1)) - A


# ---------------------------------------------------------------- hashes --

def test_hashes_match_published_finaliser(orc):
    assert fmix32(1) == 0x514E28B7  # MurmurHash3 fmix32 of 1
    for a, b in [(0, 1), (5, 9), (123456, 7654321)]:
        assert orc.pair_hash(a, b) == pair_hash(a, b)
    s = orc.level_seed(0x1234567890ABCDEF, 3)
    assert s == fmix32(0x90ABCDEF ^ fmix32((0x12345678 + 3) & 0xFFFFFFFF))
    assert orc.colour_priority(17, s) == fmix32(17 ^ s)


def test_random_start_is_splitmix(orc):
    x = orc.random_start(5, 42)
    assert np.array_equal(x, 2.0 * gen.uniform01(42, 5) - 1.0)


# ------------------------------------------------------------ validation --

def _lap(g):
    return g.laplacian()


def test_validation_accepts_both_forms(orc):
    g = gen.random_connected(30, 2)
    st, W1 = orc.input_to_adjacency(g.n, g.rowptr, g.col, g.w, True)
    rp, col, val = _lap(g)
    st2, W2 = orc.input_to_adjacency(g.n, rp, col, val, False)
    assert st == 0 and st2 == 0
    for a, b in zip(W1, W2):
        assert np.array_equal(a, b)


def test_validation_error_codes(orc):
    g = gen.random_connected(12, 3)
    rp, col, w = g.rowptr.copy(), g.col.copy(), g.w.copy()
    # asymmetric value
    w2 = w.copy()
    w2[0] += 1e-3
    assert orc.input_to_adjacency(g.n, rp, col, w2, True)[0] == orc.E_NOT_SYMMETRIC
    # negative weight in adjacency form
    w3 = w.copy()
    w3[1] = -w3[1]
    assert orc.input_to_adjacency(g.n, rp, col, w3, True)[0] == orc.E_NOT_LAPLACIAN
    # unsorted columns in a row
    c2 = col.copy()
    a = rp[0]
    c2[a], c2[a + 1] = c2[a + 1], c2[a]
    assert orc.input_to_adjacency(g.n, rp, c2, w, True)[0] == orc.E_INVALID
    # column out of range
    c3 = col.copy()
    c3[-1] = g.n
    assert orc.input_to_adjacency(g.n, rp, c3, w, True)[0] == orc.E_INVALID
    # n < 2
    assert orc.input_to_adjacency(1, np.array([0, 0]), np.zeros(0), np.zeros(0), True)[0] == \
        orc.E_INVALID
    # Laplacian with a wrong diagonal
    lrp, lcol, lval = _lap(g)
    lv = lval.copy()
    lv[np.nonzero(lcol[lrp[0]:lrp[1]] == 0)[0][0] + lrp[0]] += 1.0
    assert orc.input_to_adjacency(g.n, lrp, lcol, lv, False)[0] == orc.E_NOT_LAPLACIAN
    # isolated vertex: path 0-1 plus a vertex 2 without edges
    rp4 = np.array([0, 1, 2, 2])
    assert orc.input_to_adjacency(3, rp4, np.array([1, 0]), np.array([1.0, 1.0]), True)[0] == \
        orc.E_ISOLATED


# --------------------------------------------------------------- matching --

def _edges(n, rp, col, w):
    E = []
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            j = int(col[p])
            if j > i:
                E.append((float(w[p]), i, j))
    return E


def _key(wv, a, b):
    return (-wv, pair_hash(a, b), a, b)


def pointer_round_matching(n, rp, col, w):
    """Locally dominant matching by synchronous pointer rounds (an algorithm
    different from the oracle's sorted greedy)."""
    mate = [-1] * n
    while True:
        ptr = [-1] * n
        for v in range(n):
            if mate[v] != -1:
                continue
            best = None
            for p in range(rp[v], rp[v + 1]):
                u = int(col[p])
                if mate[u] != -1:
                    continue
                k = _key(float(w[p]), min(u, v), max(u, v))
                if best is None or k < best[0]:
                    best = (k, u)
            ptr[v] = -1 if best is None else best[1]
        active = False
        new = list(mate)
        for v in range(n):
            if mate[v] != -1:
                continue
            u = ptr[v]
            if u < 0:
                new[v] = -2
            elif ptr[u] == v:
                new[v] = u
            else:
                active = True
        mate = new
        if not active:
            return [m if m >= 0 else -1 for m in mate]


@pytest.mark.parametrize("seed", range(12))
def test_matching_equals_pointer_rounds(orc, seed):
    if seed % 3 == 0:
        g = gen.grid(6 + seed % 5, 5, "unit")  # all weights tie: the hash decides
    elif seed % 3 == 1:
        g = gen.random_connected(40 + seed, seed)
    else:
        g = gen.random_connected(30 + seed, seed, dyadic=True)  # many weight ties
    mate = orc.match(g.n, g.rowptr, g.col, g.w)
    assert list(mate) == pointer_round_matching(g.n, g.rowptr, g.col, g.w)


def test_matching_is_maximal_and_greedy(orc):
    g = gen.random_connected(60, 5)
    mate = orc.match(g.n, g.rowptr, g.col, g.w)
    E = _edges(g.n, g.rowptr, g.col, g.w)
    for wv, a, b in E:
        if mate[a] == b:
            continue
        # a non-matching edge has a matched neighbour edge that comes first
        assert mate[a] >= 0 or mate[b] >= 0
        earlier = False
        for x in (a, b):
            if mate[x] >= 0:
                y = int(mate[x])
                we = [float(g.w[p]) for p in range(g.rowptr[x], g.rowptr[x + 1]) if g.col[p] == y][0]
                if _key(we, min(x, y), max(x, y)) < _key(wv, a, b):
                    earlier = True
        assert earlier


# ------------------------------------------------------------ aggregation --

@pytest.mark.parametrize("seed", range(6))
def test_aggregation_rule(orc, seed):
    g = gen.random_connected(50 + 7 * seed, 100 + seed) if seed % 2 else gen.grid(9, 7, "unit")
    mate = orc.match(g.n, g.rowptr, g.col, g.w)
    q, nc = orc.aggregate(g.n, g.rowptr, g.col, g.w, mate)
    # independent construction of the aggregates
    root = {}
    for v in range(g.n):
        if mate[v] >= 0:
            root[v] = min(v, int(mate[v]))
    for v in range(g.n):
        if mate[v] < 0:
            best = min(((_key(float(g.w[p]), min(v, int(g.col[p])), max(v, int(g.col[p]))),
                         int(g.col[p])) for p in range(g.rowptr[v], g.rowptr[v + 1])))[1]
            root[v] = min(best, int(mate[best]))
    groups = {}
    for v in range(g.n):
        groups.setdefault(root[v], []).append(v)
    leaders = sorted(min(m) for m in groups.values())
    expect = np.zeros(g.n, np.int64)
    for members in groups.values():
        expect[members] = leaders.index(min(members))
    assert nc == len(groups)
    assert np.array_equal(q, expect)
    assert all(len(m) >= 2 for m in groups.values())
    assert nc <= g.n // 2


# --------------------------------------------------------------- Galerkin --

@pytest.mark.parametrize("seed", range(6))
def test_galerkin_equals_dense_product_exactly(orc, seed):
    g = gen.random_connected(40 + 5 * seed, 200 + seed, dyadic=True)
    mate = orc.match(g.n, g.rowptr, g.col, g.w)
    q, nc = orc.aggregate(g.n, g.rowptr, g.col, g.w, mate)
    crp, ccol, cw = orc.galerkin(g.n, g.rowptr, g.col, g.w, q, nc)
    I = np.zeros((nc, g.n))
    I[q, np.arange(g.n)] = 1.0
    Lc = I @ dense_L(g.n, g.rowptr, g.col, g.w) @ I.T
    Lo = dense_L(nc, crp, ccol, cw)
    assert np.array_equal(Lc, Lo)  # dyadic weights: every sum is exact
    for r in range(nc):
        assert np.all(np.diff(ccol[crp[r]:crp[r + 1]]) > 0)


def test_galerkin_random_weights_symmetric_bitwise(orc):
    g = gen.random_connected(300, 9)
    mate = orc.match(g.n, g.rowptr, g.col, g.w)
    q, nc = orc.aggregate(g.n, g.rowptr, g.col, g.w, mate)
    crp, ccol, cw = orc.galerkin(g.n, g.rowptr, g.col, g.w, q, nc)
    Wc = dense_W(nc, crp, ccol, cw)
    assert np.array_equal(Wc, Wc.T)
    I = np.zeros((nc, g.n))
    I[q, np.arange(g.n)] = 1.0
    Lc = I @ dense_L(g.n, g.rowptr, g.col, g.w) @ I.T
    W_expect = np.diag(np.diag(Lc)) - Lc
    assert np.allclose(Wc, W_expect, rtol=1e-14, atol=1e-14)


# -------------------------------------------------------------- colouring --

def jones_plassmann(n, rp, col, seed):
    """Parallel rounds: colour a vertex once all higher-priority neighbours are
    coloured (an algorithm different from the oracle's sorted first-fit)."""
    pr = [fmix32(v ^ seed) for v in range(n)]
    colour = [-1] * n
    while -1 in colour:
        snap = list(colour)
        for v in range(n):
            if snap[v] >= 0:
                continue
            nb = [int(col[p]) for p in range(rp[v], rp[v + 1])]
            if any(snap[u] < 0 and (pr[u] > pr[v] or (pr[u] == pr[v] and u < v)) for u in nb):
                continue
            used = {snap[u] for u in nb if snap[u] >= 0}
            c = 0
            while c in used:
                c += 1
            colour[v] = c
    return colour


@pytest.mark.parametrize("seed", range(6))
def test_colouring_equals_jones_plassmann(orc, seed):
    g = gen.random_connected(60 + seed, 300 + seed) if seed % 2 else gen.grid(8, 6 + seed)
    s = orc.level_seed(seed, seed)
    c, k = orc.colour(g.n, g.rowptr, g.col, s)
    assert list(c) == jones_plassmann(g.n, g.rowptr, g.col, s)
    assert k == max(c) + 1
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    assert np.all(c[rows] != c[g.col])  # proper colouring
    assert k <= np.diff(g.rowptr).max() + 1


def iterated_greedy(n, rp, col, colour):
    """Classes from the highest colour down; inside a class every vertex
    chooses at once from a snapshot of the colours already assigned (a class
    is an independent set, so this is the sequential pass done in rounds)."""
    colour = np.asarray(colour)
    new = np.full(n, -1)
    for c in range(int(colour.max()), -1, -1):
        snap = new.copy()
        for v in np.nonzero(colour == c)[0]:
            used = {int(snap[u]) for u in col[rp[v]:rp[v + 1]] if snap[u] >= 0}
            k = 0
            while k in used:
                k += 1
            new[v] = k
    return new


def test_recolouring_path_closed_form(orc):
    # path a-b-c-d coloured 0,1,2,0 (first-fit in the order a, d, b, c): the
    # pass takes c first (colour 0), then b (1), then a and d -> 2 colours
    g = gen.path(4)
    c, k = orc.recolour(4, g.rowptr, g.col, [0, 1, 2, 0], 3)
    assert list(c) == [0, 1, 0, 1] and k == 2


@pytest.mark.parametrize("seed", range(6))
def test_recolouring_equals_class_rounds(orc, seed):
    g = gen.random_connected(60 + seed, 300 + seed) if seed % 2 else gen.grid(8, 6 + seed)
    c0, k0 = orc.colour(g.n, g.rowptr, g.col, orc.level_seed(seed, seed))
    c, k = orc.recolour(g.n, g.rowptr, g.col, c0, k0)
    assert list(c) == list(iterated_greedy(g.n, g.rowptr, g.col, c0))
    assert k == max(c) + 1 and k <= k0
    assert set(c) == set(range(k))  # first-fit leaves no gaps
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    assert np.all(c[rows] != c[g.col])


def bfs_parity_colouring(n, rp, col):
    """Independent two-colouring: unweighted distances from each connected
    component's smallest vertex (scipy's breadth-first shortest paths), taken
    mod 2; None when an edge joins equal parities (an odd cycle)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components, shortest_path

    A = sp.csr_matrix((np.ones(len(col)), col, rp), shape=(n, n))
    ncomp, lab = connected_components(A, directed=False)
    out = np.zeros(n, np.int64)
    for c in range(ncomp):
        members = np.nonzero(lab == c)[0]
        d = shortest_path(A, unweighted=True, directed=False, indices=int(members.min()))
        out[members] = d[members].astype(np.int64) % 2
    rows = np.repeat(np.arange(n), np.diff(rp))
    if np.any(out[rows] == out[col]):
        return None
    return out


def _cycle(n):
    a = np.arange(n)
    return gen._csr_from_undirected(n, a, (a + 1) % n, np.ones(n))


def test_two_colouring_closed_forms(orc):
    # grid r x c, vertex id r*cols + c: the checkerboard (r + c) mod 2
    g = gen.grid(7, 5)
    c, k = orc.colour_two(g.n, g.rowptr, g.col)
    r, cc = np.divmod(np.arange(g.n), 5)
    assert k == 2 and np.array_equal(c, (r + cc) % 2)
    # path: alternating from vertex 0
    g = gen.path(9)
    c, k = orc.colour_two(g.n, g.rowptr, g.col)
    assert k == 2 and list(c) == [i % 2 for i in range(9)]
    # even cycle is bipartite, odd cycle is not
    g = _cycle(8)
    assert orc.colour_two(g.n, g.rowptr, g.col)[1] == 2
    g = _cycle(9)
    assert orc.colour_two(g.n, g.rowptr, g.col)[1] == 0


def _random_bipartite(n, seed, with_odd_edge=False):
    u = gen.uniform01(seed, 4 * n)
    side = (u[:n] < 0.5).astype(int)
    side[0], side[1] = 0, 1
    a, b = [], []
    for k in range(n - 1):  # a spanning path that alternates when possible
        i, j = k, k + 1
        a.append(i)
        b.append(j)
    pairs = set()
    idx = (u[n:] * n).astype(int)
    for k in range(0, len(idx) - 1, 2):
        i, j = int(idx[k]), int(idx[k + 1])
        if i != j and (side[i] != side[j]):
            pairs.add((min(i, j), max(i, j)))
    # the spanning path may join equal sides: keep only cross edges plus a
    # cross-side chain so that the graph stays bipartite and connected
    lo = [v for v in range(n) if side[v] == 0]
    hi = [v for v in range(n) if side[v] == 1]
    for k in range(max(len(lo), len(hi))):
        x, y = lo[min(k, len(lo) - 1)], hi[min(k, len(hi) - 1)]
        pairs.add((min(x, y), max(x, y)))
    if with_odd_edge:
        pairs.add((lo[0], lo[1]) if lo[0] < lo[1] else (lo[1], lo[0]))
    pairs = sorted(pairs)
    a = np.array([p[0] for p in pairs])
    b = np.array([p[1] for p in pairs])
    return gen._csr_from_undirected(n, a, b, np.ones(len(a)))


@pytest.mark.parametrize("seed", range(6))
def test_two_colouring_equals_bfs_parity(orc, seed):
    """Random bipartite graphs (and, for odd seeds, the same with one edge
    inside a side): the oracle's two-colouring equals the distance parity from
    each component's smallest vertex, and an odd cycle is reported as 0."""
    g = _random_bipartite(50 + 7 * seed, 900 + seed, with_odd_edge=seed % 2 == 1)
    c, k = orc.colour_two(g.n, g.rowptr, g.col)
    ref = bfs_parity_colouring(g.n, g.rowptr, g.col)
    if ref is None:
        assert k == 0
    else:
        assert k == 2 and np.array_equal(c, ref)
    # a disconnected bipartite graph: two paths side by side
    a = np.array([0, 1, 3, 4, 5])
    b = np.array([1, 2, 4, 5, 6])
    g2 = gen._csr_from_undirected(7, a, b, np.ones(5))
    c2, k2 = orc.colour_two(7, g2.rowptr, g2.col)
    assert k2 == 2 and list(c2) == [0, 1, 0, 0, 1, 0, 1]


@pytest.mark.parametrize("kind", ["grid", "path", "rgg"])
def test_hierarchy_colourings(orc, kind):
    """The finest level's colouring is its two-colouring when it is bipartite
    (grids, paths); every other level's, and a non-bipartite finest level's,
    is first-fit in priority order followed by one iterated-greedy pass."""
    g = {"grid": lambda: gen.grid(40, 30, "uniform", seed=6), "path": lambda: gen.path(200),
         "rgg": lambda: gen.rgg(3000, 4)}[kind]()
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=8, colour_seed=5)
    for l in range(h.nlevels - 1):
        L = h.level(l)
        ref = bfs_parity_colouring(L.n, L.rowptr, L.col) if l == 0 else None
        if l == 0:
            assert (ref is None) == (kind == "rgg")
        if ref is not None:
            assert np.array_equal(L.colour, ref) and L.ncolours == 2, l
            continue
        c0 = jones_plassmann(L.n, L.rowptr, L.col, orc.level_seed(5, l))
        c = iterated_greedy(L.n, L.rowptr, L.col, c0)
        assert np.array_equal(L.colour, c), l
        assert L.ncolours == c.max() + 1


# ------------------------------------------------------ smoother and power --

def _colour_order(c):
    return np.lexsort((np.arange(len(c)), c))


@pytest.mark.parametrize("omega", [1.0, 1.5])
@pytest.mark.parametrize("rho", [0.05, 3.0])
def test_gs_sweep_is_matrix_splitting(orc, omega, rho):
    # rho = 3 exceeds the degree of some rows: no row is special-cased
    g = gen.random_connected(48, 17)
    c, k = orc.colour(g.n, g.rowptr, g.col, orc.level_seed(0, 0))
    x = np.sin(np.arange(g.n) * 0.7)
    W = dense_W(g.n, g.rowptr, g.col, g.w)
    d = W.sum(1)
    assert d.min() < rho or rho < 1
    o = _colour_order(c)
    Wp = W[np.ix_(o, o)]
    Dp = np.diag(d[o])
    Wl, Wu = np.tril(Wp, -1), np.triu(Wp, 1)
    # SOR on the splitting L - rho I = (D - W_l) - (W_u + rho I):
    # (D - omega W_l) x' = ((1 - omega) D + omega (W_u + rho I)) x
    xp = np.linalg.solve(Dp - omega * Wl,
                         ((1 - omega) * Dp + omega * (Wu + rho * np.eye(g.n))) @ x[o])
    expect = np.empty(g.n)
    expect[o] = xp
    got = oracle_sweep(orc, g, c, k, x, rho, omega)
    assert np.allclose(got, expect, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("rho", [0.0, 0.05, 3.0])
def test_lexicographic_sweep_is_matrix_splitting(orc, rho):
    """Algorithm 2's literal order (rows 1..n, the oracle-only mode): one sweep
    solves (D - W_l) x' = (W_u + rho I) x with W_l / W_u the strict lower /
    upper triangles in the natural index order (no permutation)."""
    g = gen.random_connected(40, 29)
    x = np.cos(np.arange(g.n) * 0.31) + 0.1
    W = dense_W(g.n, g.rowptr, g.col, g.w)
    D = np.diag(W.sum(1))
    Wl, Wu = np.tril(W, -1), np.triu(W, 1)
    expect = np.linalg.solve(D - Wl, (Wu + rho * np.eye(g.n)) @ x)
    got = orc.gs_sweep_lex(g.n, g.rowptr, g.col, g.w, x.copy(), rho=rho)
    assert np.allclose(got, expect, rtol=1e-13, atol=1e-13)
    # one sweep differs from the multicolour order's on the same graph: the
    # order matters, so a wrong row range would show
    c, k = orc.colour(g.n, g.rowptr, g.col, orc.level_seed(0, 0))
    assert not np.allclose(oracle_sweep(orc, g, c, k, x, rho, 1.0), expect, atol=1e-6)


@pytest.mark.parametrize("k", [24, 40])
def test_lexicographic_mode_solves_path(orc, k):
    """The whole solve in the lexicographic order on a path of k vertices: the
    closed form lambda_2 = 2 - 2 cos(pi/k), phi_2 = cos(pi (i + 1/2)/k)."""
    g = gen.path(k)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=4)
    r = h.solve(seed=1, lexicographic=True, tol_cos=1e-14, tol_res=1e-11, max_gs=2000,
                max_pi=20, max_outer=20000)
    lam = 2 - 2 * math.cos(math.pi / k)
    assert r.status == 0 and abs(r.lam - lam) <= 1e-10 * lam
    phi = np.cos(math.pi * (np.arange(k) + 0.5) / k)
    phi /= np.linalg.norm(phi)
    assert 1 - abs(float(r.x @ phi)) <= 1e-9
    # the lexicographic schedule is not the multicolour one
    rm = h.solve(seed=1, tol_cos=1e-14, tol_res=1e-11, max_gs=2000, max_pi=20, max_outer=20000)
    assert r.counts != rm.counts or r.x.tobytes() != rm.x.tobytes()


def oracle_sweep(orc, g, c, k, x, rho, omega):
    import ctypes as C
    xx = np.ascontiguousarray(x, dtype=np.float64).copy()
    orc.lib().or_gs_sweep(g.n, g.rowptr, g.col, g.w, np.ascontiguousarray(c, np.int32), k, rho,
                          omega, xx)
    return xx


def test_fiedler_vector_is_fixed_point_of_shifted_sweep(orc):
    g = gen.grid(12, 10, "uniform", seed=1)
    L = dense_L(g.n, g.rowptr, g.col, g.w)
    ev, V = np.linalg.eigh(L)
    phi = V[:, 1]
    c, k = orc.colour(g.n, g.rowptr, g.col, 7)
    out = oracle_sweep(orc, g, c, k, phi, ev[1], 1.0)
    assert np.allclose(out, phi, atol=1e-12)
    # the unshifted sweep of the b = 0 reading does not keep it (non-regular graph)
    out0 = oracle_sweep(orc, g, c, k, phi, 0.0, 1.0)
    assert np.linalg.norm(orc.project_normalise(out0) - phi) > 1e-3
    # the all-ones vector is a fixed point of the unshifted sweep
    one = np.ones(g.n)
    assert np.allclose(oracle_sweep(orc, g, c, k, one, 0.0, 1.0), one, atol=1e-15)


def test_power_step_and_sigma(orc):
    g = gen.random_connected(30, 4)
    L = dense_L(g.n, g.rowptr, g.col, g.w)
    sig = orc.sigma(g.n, g.rowptr, g.w)
    def row_sum(i):  # sequential, in row order
        s = 0.0
        for v in g.w[g.rowptr[i]:g.rowptr[i + 1]]:
            s += float(v)
        return s

    assert sig == 2.0 * max(row_sum(i) for i in range(g.n))
    assert sig >= np.linalg.eigvalsh(L).max()  # Gershgorin: B = sigma I - L >= 0
    x = np.cos(np.arange(g.n))
    assert np.allclose(orc.pi_apply(g.n, g.rowptr, g.col, g.w, sig, x), sig * x - L @ x,
                       rtol=1e-14, atol=1e-13)


def test_rayleigh_and_residual_dense(orc):
    g = gen.random_connected(35, 8)
    L = dense_L(g.n, g.rowptr, g.col, g.w)
    x = np.sin(np.arange(g.n) * 1.3) + 0.2
    rho, res = orc.rq_residual(g.n, g.rowptr, g.col, g.w, x)
    r_exp = x @ L @ x / (x @ x)
    assert abs(rho - r_exp) <= 1e-14 * abs(r_exp)
    assert abs(res - np.linalg.norm(L @ x - r_exp * x) / np.linalg.norm(x)) < 1e-13


# --------------------------------------------------------------- coarsest --

@pytest.mark.parametrize("seed", range(5))
def test_coarsest_power_iteration_vs_eigh(orc, seed):
    g = gen.random_connected(8 + 4 * seed, 50 + seed)
    L = dense_L(g.n, g.rowptr, g.col, g.w)
    ev, V = np.linalg.eigh(L)
    sig = orc.sigma(g.n, g.rowptr, g.w)
    x, it, conv = orc.coarsest(g.n, g.rowptr, g.col, g.w, sig, seed + 1)
    assert conv
    lam = x @ L @ x
    assert abs(lam - ev[1]) <= 1e-12 * max(1.0, ev[1])
    if ev[2] - ev[1] > 1e-3:
        assert 1 - abs(x @ V[:, 1]) <= 1e-12
    assert abs(x.sum()) < 1e-12 and abs(np.linalg.norm(x) - 1) < 1e-14


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-9])
def test_coarsest_stops_at_first_step_below_tolerance(orc, tol):
    """The stop rule: the returned iterate is the first whose residual
    ||L x - (x^T L x) x|| is at or below tol * sigma; the iterate one step
    earlier (rerun with a forced count) is above it, and the residuals are
    recomputed here from the dense Laplacian."""
    g = gen.random_connected(20, 71)
    L = dense_L(g.n, g.rowptr, g.col, g.w)
    sig = orc.sigma(g.n, g.rowptr, g.w)

    def res(v):
        return np.linalg.norm(L @ v - (v @ L @ v) * v)

    x, it, conv = orc.coarsest(g.n, g.rowptr, g.col, g.w, sig, 3, tol=tol)
    assert conv and it > 0
    assert res(x) <= tol * sig * (1 + 1e-9)
    xp, itp, _ = orc.coarsest(g.n, g.rowptr, g.col, g.w, sig, 3, replay_it=it - 1)
    assert itp == it - 1 and res(xp) > tol * sig * (1 - 1e-9)
    _, it_tight, _ = orc.coarsest(g.n, g.rowptr, g.col, g.w, sig, 3)
    assert it_tight > it


# ------------------------------------------------------------ whole solve --

TIGHT = dict(tol_cos=1e-10, tol_res=1e-9, max_gs=2000, max_pi=50, max_outer=20000)


def test_paper_square_grid_within_kato_temple(orc):
    """The smallest square grid of the paper's scaling table (326 x 326 = 106,276
    vertices, unit weights) with the parameters of the square-grid scaling
    workload (SOR factor 1.95 on the red-black finest level): residual <= 1e-6,
    and the eigenvalue within the Kato-Temple bound r^2 / (lambda_next -
    lambda) of the double eigenvalue 2 - 2 cos(pi/326), the next distinct one
    being twice that."""
    k = 326
    g = gen.grid(k, k)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
    assert h.level(0).ncolours == 2
    r = h.solve(seed=1, tol_cos=3e-12, tol_res=1e-6, omega=1.95, max_gs=30, max_pi=1,
                max_outer=400, tol_coarse=1e-6)
    lam2 = 2 - 2 * math.cos(math.pi / k)
    assert r.status == 0 and r.residual <= 1e-6
    assert abs(r.lam - lam2) <= r.residual ** 2 / (2 * lam2 - r.lam)


@pytest.mark.parametrize("n", [2, 3, 5, 9, 16, 33, 64])
def test_path_closed_form(orc, n):
    g = gen.path(n)
    h, r = orc.solve_graph(g, n_coarse=8, **TIGHT)
    lam = 2.0 - 2.0 * math.cos(math.pi / n)
    assert r.status == 0
    assert abs(r.lam - lam) <= 1e-9 * lam
    phi = np.cos(math.pi * (np.arange(n) + 0.5) / n)
    phi /= np.linalg.norm(phi)
    assert 1 - abs(r.x @ phi) <= 1e-8
    assert r.x[0] > 0  # sign convention: first significant entry positive


@pytest.mark.parametrize("m,k", [(32, 24), (12, 7), (20, 9)])
def test_grid_closed_form(orc, m, k):
    g = gen.grid(m, k)
    h, r = orc.solve_graph(g, n_coarse=8, **TIGHT)
    lam = 2.0 - 2.0 * math.cos(math.pi / max(m, k))
    assert r.status == 0
    assert abs(r.lam - lam) <= 1e-9 * lam
    if (m, k) == (32, 24):
        assert abs(lam - 0.009630546655606143) < 1e-17


@pytest.mark.parametrize("seed", range(4))
def test_random_graph_vs_eigh(orc, seed):
    g = gen.random_connected(64, 900 + seed)
    ev, V = np.linalg.eigh(dense_L(g.n, g.rowptr, g.col, g.w))
    h, r = orc.solve_graph(g, n_coarse=8, **TIGHT)
    assert r.status == 0
    # residual bound (Kato-Temple): |rho - lambda_2| <= r^2 / (lambda_3 - rho)
    assert abs(r.lam - ev[1]) <= r.residual ** 2 / (ev[2] - r.lam) + 1e-12
    assert abs(r.lam - ev[1]) <= 1e-9 * ev[1]


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("omega", [1.0, 1.9])
def test_erdos_renyi_with_pendants_vs_eigh(orc, seed, omega):
    # expander-like graph whose lambda_2 is comparable to its smallest degrees:
    # the shift then exceeds the degree of some rows, and the sweep must still
    # converge to phi_2 (over-relaxed too)
    g = gen.erdos_renyi(400, 6 / 399, 100 + seed)
    L = dense_L(g.n, g.rowptr, g.col, g.w)
    ev = np.linalg.eigvalsh(L)
    assert np.diag(L).min() < 2 * ev[1]
    h, r = orc.solve_graph(g, n_coarse=8, omega=omega, **TIGHT)
    assert r.status == 0
    assert abs(r.lam - ev[1]) <= r.residual ** 2 / (ev[2] - r.lam) + 1e-12
    assert abs(r.lam - ev[1]) <= 1e-9 * ev[1]


def test_large_grid_courant_fischer_vs_eigsh(orc):
    from scipy.sparse.linalg import eigsh

    g = gen.grid(200, 150, "uniform", seed=2)
    A = csr_matrix((g.w, g.col, g.rowptr), shape=(g.n, g.n))
    L = (csr_matrix(np.diag(np.asarray(A.sum(1)).ravel())) - A).tocsc()
    vals = eigsh(L, k=3, sigma=-1e-3, which="LM", return_eigenvectors=False)
    lam2, lam3 = sorted(vals)[1], sorted(vals)[2]
    h, r = orc.solve_graph(g, n_coarse=25, tol_cos=1e-12, max_gs=2000, max_pi=5)
    assert r.lam >= lam2 - 1e-15  # Courant-Fischer: x orthogonal to ones
    assert r.lam - lam2 <= r.residual ** 2 / (lam3 - r.lam) + 1e-15
    assert abs(r.x.sum()) < 1e-10 and abs(np.linalg.norm(r.x) - 1) < 1e-12


# ------------------------------------------------------ hierarchy invariants --

@pytest.mark.parametrize("which", ["grid", "rgg", "er", "rand"])
def test_hierarchy_invariants(orc, which):
    g = {"grid": gen.grid(40, 30, "uniform", seed=1), "rgg": gen.rgg(3000, 4),
         "er": gen.erdos_renyi(2000, 6 / 1999, 6), "rand": gen.random_connected(500, 3)}[which]
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=10)
    tot = g.w.sum()
    for l in range(h.nlevels):
        L = h.level(l)
        W = csr_matrix((L.w, L.col, L.rowptr), shape=(L.n, L.n))
        assert (W != W.T).nnz == 0 and np.all(L.w > 0)
        assert connected_components(W, directed=False)[0] == 1
        assert np.all(np.diff(L.rowptr) > 0)  # no isolated vertex
        if l + 1 < h.nlevels:
            assert h.level(l + 1).n <= L.n // 2
            q = L.q
            rows = np.repeat(np.arange(L.n), np.diff(L.rowptr))
            inner = L.w[q[rows] == q[L.col]].sum()
            assert abs(h.level(l + 1).w.sum() - (L.w.sum() - inner)) <= 1e-9 * tot
    assert h.level(h.nlevels - 1).n <= 10


def test_replay_reproduces_schedule_bitwise(orc):
    g = gen.grid(30, 20, "uniform", seed=5)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=8)
    r1 = h.solve(seed=3)
    r2 = h.solve(seed=3, replay=r1.counts)
    assert r2.counts == r1.counts
    assert np.array_equal(r1.x, r2.x) and r1.lam == r2.lam


# ------------------------------------------- randomised heavy edge coarsening --

def hec_reference(n, rp, col, w, perm):
    """Algorithm 1 written out in Python on a dense copy: in the visiting order,
    an unassigned vertex takes the smallest entry of its column of L
    (argmin over the whole column, the diagonal included: the most negative
    entry is the heaviest edge; the first index on ties) and pairs with it or
    joins its aggregate."""
    Ld = -dense_W(n, rp, col, w)
    np.fill_diagonal(Ld, -Ld.sum(axis=1))
    q = np.full(n, -1)
    c = 0
    for v in perm:
        if q[v] >= 0:
            continue
        m = int(np.argmin(Ld[:, v]))
        if q[m] < 0:
            q[m] = q[v] = c
            c += 1
        else:
            q[v] = q[m]
    return q, c


@pytest.mark.parametrize("seed", range(5))
def test_randomised_hec_equals_algorithm_1(orc, seed):
    g = gen.random_connected(70 + 9 * seed, 500 + seed, dyadic=seed % 2 == 0)
    perm = orc.randperm(g.n, 99 + seed)
    assert sorted(perm) == list(range(g.n))
    q, c = orc.hec_random(g.n, g.rowptr, g.col, g.w, perm)
    qr, cr = hec_reference(g.n, g.rowptr, g.col, g.w, perm)
    assert c == cr and np.array_equal(q, qr)
    sizes = np.bincount(q, minlength=c)
    assert sizes.min() >= 2 and c <= g.n // 2  # every aggregate has two or more vertices


def test_randomised_hec_hierarchy_solves_grid(orc):
    """The whole method on hierarchies from the paper's randomised coarsening:
    the 20 x 9 grid's lambda_2 = 2 - 2 cos(pi/20), and each level at most half
    the previous one."""
    g = gen.grid(20, 9)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=8, hec_seed=7)
    ns = [h.level(l).n for l in range(h.nlevels)]
    assert all(b <= a // 2 for a, b in zip(ns, ns[1:]))
    r = h.solve(seed=1, tol_cos=1e-12, tol_res=1e-10, max_gs=2000, max_pi=20, max_outer=5000)
    lam = 2 - 2 * math.cos(math.pi / 20)
    assert r.status == 0 and abs(r.lam - lam) <= 1e-9 * lam


# ------------------------------------------- smoother and coarse-problem variants --

def _eig2(g):
    W = dense_W(g.n, g.rowptr, g.col, g.w)
    L = np.diag(W.sum(1)) - W
    vals, vecs = np.linalg.eigh(L)
    return vals, vecs


@pytest.mark.parametrize("variant", [dict(coarse_mass=True), dict(lanczos_k=8),
                                     dict(max_gs=0, max_pi=400)])
@pytest.mark.parametrize("seed", [3, 4])
def test_variants_reach_lambda_2(orc, variant, seed):
    """Every oracle variant of the smoother or the coarse problems, run to a
    tight residual, ends at lambda_2 of a random 64-vertex graph (numpy eigh),
    its vector within the Kato-Temple-style angle bound."""
    g = gen.random_connected(64, 800 + seed)
    vals, vecs = _eig2(g)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=6)
    kw = dict(seed=1, tol_cos=1e-14, tol_res=1e-10, max_gs=400, max_pi=5, max_outer=20000)
    kw.update(variant)
    r = h.solve(**kw)
    assert r.status == 0 and r.residual <= 1e-10
    gap = vals[2] - vals[1]
    assert abs(r.lam - vals[1]) <= r.residual ** 2 / gap * 1.01 + 1e-14
    assert 1 - abs(float(r.x @ vecs[:, 1])) <= (r.residual / gap) ** 2 + 1e-12


def test_lanczos_phase_exact_in_full_krylov_space(orc):
    """n - 1 Lanczos steps span the whole complement of 1, so the top Ritz
    vector of sigma I - L is phi_2 exactly (random 30-vertex graph)."""
    g = gen.random_connected(30, 812)
    vals, vecs = _eig2(g)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=2)
    # one level above the coarsest: replay a single Lanczos phase of n-1 steps
    # on level 0 after the cascade, then compare
    J = h.nlevels - 1
    r = h.solve(seed=1, lanczos_k=29, replay=[0] + [0, 0] * (J - 1) + [29, 0])
    assert 1 - abs(float(r.x @ vecs[:, 1])) <= 1e-10
    assert abs(r.lam - vals[1]) <= 1e-10 * vals[1]


def test_mass_weighted_coarse_problem_is_ritz_projection(orc):
    """On one coarsening, the mass-weighted coarse problem's smallest nonzero
    eigenvalue equals the Ritz value of L on the aggregates' indicator vectors
    (min over y of (I^T y)^T L (I^T y) / (I^T y)^T (I^T y)), and its masses are
    the aggregate sizes."""
    import scipy.linalg as sl

    g = gen.random_connected(40, 813)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=30)
    L0, L1 = h.level(0), h.level(1)
    P = np.zeros((L0.n, L1.n))
    P[np.arange(L0.n), L0.q] = 1.0
    W = dense_W(g.n, g.rowptr, g.col, g.w)
    L = np.diag(W.sum(1)) - W
    ritz = sl.eigh(P.T @ L @ P, P.T @ P, eigvals_only=True)
    Wc = dense_W(L1.n, L1.rowptr, L1.col, L1.w)
    Lc = np.diag(Wc.sum(1)) - Wc
    M = np.diag(np.bincount(L0.q, minlength=L1.n).astype(float))
    gen_vals = sl.eigh(Lc, M, eigvals_only=True)
    assert np.allclose(gen_vals, ritz, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", [3, 4])
def test_rhs_y_reading_does_not_converge(orc, seed):
    """The reading of Algorithm 3's GS(L, y) with right-hand side b = y (the
    iterate before the sweep) has the fixed points of (L - I) x = 0, not
    phi_2: on the same graphs as above it stalls with a residual above 1e-2,
    which is why the library's sweep takes the Rayleigh shift instead."""
    g = gen.random_connected(64, 800 + seed)
    h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=6)
    r = h.solve(seed=1, tol_cos=1e-14, tol_res=1e-10, max_gs=400, max_pi=5, max_outer=2000,
                rhs_y=True)
    assert r.status == orc.E_NOT_CONVERGED and r.residual > 1e-2


# --------------------------------------------------------------------------
# Spectral partitioning (recursive bisection of phi_2, the application the
# Introduction names): the oracle's recursion against closed forms.
# --------------------------------------------------------------------------

PART_KW = dict(seed=1, tol_cos=1e-12, tol_res=1e-9, max_gs=200, max_pi=10, max_outer=400)


@pytest.mark.parametrize("parts", [2, 4, 8])
def test_partition_of_path_is_intervals(orc, parts):
    """phi_2 of a path is cos(pi (i + 1/2) / n), strictly monotone, and every
    part of a median cut is again a path: each of the parts must be an
    interval of n / parts consecutive vertices, and the cut weight is the
    parts - 1 edges between them."""
    n = 64
    g = gen.path(n)
    labels, n_iso = orc.spectral_partition(g, parts, "median", **PART_KW)
    assert n_iso == 0
    size = n // parts
    blocks = labels.reshape(parts, size)
    assert (blocks == blocks[:, :1]).all()  # constant on each interval
    assert sorted(blocks[:, 0].tolist()) == list(range(parts))


def test_partition_of_path_sign_cut_halves(orc):
    """phi_2 of an even path changes sign exactly between n/2 - 1 and n/2."""
    g = gen.path(40)
    labels, _ = orc.spectral_partition(g, 2, "sign", **PART_KW)
    assert len(set(labels[:20].tolist())) == 1 and len(set(labels[20:].tolist())) == 1
    assert labels[0] != labels[-1]


def test_partition_of_long_grid_cuts_across_the_long_side(orc):
    """On a 4 x 16 unit grid lambda_2 = 2 - 2 cos(pi / 16) belongs to
    cos(pi (c + 1/2) / 16), constant down each column; each half (4 x 8) has
    lambda_2 = 2 - 2 cos(pi / 8) < 2 - 2 cos(pi / 4) again along its long side.
    So four median parts are the column blocks 0-3, 4-7, 8-11 and 12-15, and
    the cut is 3 x 4 unit edges."""
    g = gen.grid(4, 16)
    labels, _ = orc.spectral_partition(g, 4, "median", **PART_KW)
    lab = labels.reshape(4, 16)
    assert (lab == lab[:1]).all()  # every row cut the same way
    cols = lab[0].reshape(4, 4)
    assert (cols == cols[:, :1]).all() and sorted(cols[:, 0].tolist()) == [0, 1, 2, 3]
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    cut = (labels[rows] != labels[g.col]) & (g.col > rows)
    assert float(g.w[cut].sum()) == 12.0


def test_partition_separates_two_cliques(orc):
    """Two 8-cliques joined by one edge: phi_2 is positive on one clique and
    negative on the other (it is constant on each clique apart from the two
    endpoints of the bridge, which keep the sign of their clique), so both
    cuts give the cliques, with cut weight 1."""
    a, b = [], []
    for base in (0, 8):
        for i in range(8):
            for j in range(i + 1, 8):
                a.append(base + i)
                b.append(base + j)
    a.append(7)
    b.append(8)
    g = gen._csr_from_undirected(16, np.array(a), np.array(b), np.ones(len(a)))
    for cut in ("median", "sign"):
        labels, _ = orc.spectral_partition(g, 2, cut, **PART_KW)
        assert len(set(labels[:8].tolist())) == 1 and len(set(labels[8:].tolist())) == 1
        assert labels[0] != labels[8]


def test_partition_isolated_vertex_rule_worked_example(orc):
    """A worked example of the rules for vertices left without an edge inside
    their part: path 0-1-2-3 with a pendant 4 on vertex 0, and a supplied
    vector equal to the vertex index. Round 1 (median): {0, 1} -> 0,
    {2, 3, 4} -> 1. Round 2: part 0 splits into {0} -> 0 and {1} -> 1; in part
    1 vertex 4 has no neighbour, {2} -> 2, {3} -> 3, and 4 joins the smaller
    half, 2 on the tie. Labels [0, 1, 2, 3, 2], one isolated vertex."""
    g = gen._csr_from_undirected(5, np.array([0, 1, 2, 0]), np.array([1, 2, 3, 4]), np.ones(4))
    labels, n_iso = orc.spectral_partition(
        g, 4, "median", vector=lambda sub: np.arange(sub.n, dtype=np.float64))
    assert labels.tolist() == [0, 1, 2, 3, 2] and n_iso == 1


def test_zero_cosine_tolerance_runs_every_phase_to_its_cap(orc):
    """tol_cos <= 0 switches the cosine stop off (Section 4's test compares
    the cosine of successive unit iterates with 1 - tol_cos; against exactly 1
    it could fire on rounding once the iterates agree to the last bit): every
    phase then runs its full sweep and step caps, so the schedule is the caps
    alone, also for many power steps on a graph where they converge fast."""
    for g, nc in ((gen.grid(20, 9), 8), (gen.random_connected(64, 802), 6)):
        h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
        J = h.nlevels - 1
        r = h.solve(seed=1, tol_cos=0.0, max_gs=7, max_pi=40, tol_res=1e-30, max_outer=3)
        assert r.counts[1:] == [7, 40] * (J + 3)


def _reaches(res, res_prev, tol, left):
    """Closed form of the early-exit test: a residual falling by q = res /
    res_prev per round reaches tol within `left` rounds iff the rounds it
    needs, ceil(log(tol / res) / log q), are at most `left`."""
    if not res < res_prev:
        return False
    if res <= tol:
        return True
    return math.ceil(math.log(tol / res) / math.log(res / res_prev)) <= left


def test_early_exit_rule_against_its_closed_form(orc):
    """or_can_reach (round-by-round products) against the logarithmic closed
    form, on cases kept away from ties, and its answers when the residual did
    not fall."""
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(3000):
        res, q = 10 ** rng.uniform(-6, -3), rng.uniform(0.3, 0.999)
        left, tol = int(rng.integers(0, 60)), 1e-6
        need = math.log(tol / res) / math.log(q)
        if res <= tol or abs(need - round(need)) < 1e-6:
            continue
        assert orc.can_reach(res, res / q, tol, left) == (math.ceil(need) <= left), (res, q, left)
        checked += 1
    assert checked > 1500
    assert not orc.can_reach(2e-6, 2e-6, 1e-6, 400)  # no fall
    assert not orc.can_reach(2e-6, 1e-6, 1e-6, 400)  # a rise


# Serving-pool parameters: long phases, no cosine stop, SOR 1.95, 12 rounds.
SERVE_PARAMS = dict(seed=1, tol_cos=0.0, tol_res=1e-6, max_gs=30, max_pi=30, omega=1.95,
                    max_outer=12, tol_coarse=1e-6)


def test_early_exit_stops_where_the_rule_says(orc):
    """With early exit the oracle's finest rounds end at the first round whose
    residual, against the one before it, fails the closed-form test (the
    trajectory taken from the same solve run for 0, 1, 2, ... rounds without
    early exit), and return that round's residual; a graph that converges
    within the cap runs as without early exit."""
    for n, seed, stalls in ((1523, gen.derive_seed(5, 22) ^ 0x55, True), (3000, 11, False)):
        g = gen.rgg(n, seed)
        h = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
        J = h.nlevels - 1
        P = dict(SERVE_PARAMS)
        traj = [h.solve(**dict(P, max_outer=k)).residual for k in range(P["max_outer"] + 1)]
        expect = P["max_outer"]
        for k in range(1, P["max_outer"] + 1):
            if traj[k] <= P["tol_res"] or not _reaches(traj[k], traj[k - 1], P["tol_res"],
                                                       P["max_outer"] - k):
                expect = k
                break
        r = h.solve(early_exit=True, **P)
        rounds = (len(r.counts) - 1 - 2 * J) // 2
        assert rounds == expect and r.residual == traj[expect], (n, rounds, expect)
        assert (rounds < P["max_outer"]) == stalls
        r0 = h.solve(**P)
        if not stalls:
            assert r0.counts == r.counts and r0.residual == r.residual
