"""Input generators: published SplitMix64 values and the structure of every
graph family (symmetric CSR, sorted columns, connected where promised)."""
import math
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import gen


def test_splitmix64_published_values():
    # SplitMix64 seeded with 0 (Vigna's reference C code): first three outputs.
    z = gen.splitmix64(0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform01_range():
    u = gen.uniform01(7, 10000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01


def _check_csr(g, connected=True):
    assert g.rowptr[0] == 0 and g.rowptr[-1] == g.m
    assert np.all(np.diff(g.rowptr) >= 0)
    A = csr_matrix((g.w, g.col, g.rowptr), shape=(g.n, g.n))
    for i in range(0, g.n, max(1, g.n // 50)):
        c = g.col[g.rowptr[i]:g.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0) and not np.any(c == i)
    assert (A != A.T).nnz == 0
    assert np.all(g.w > 0)
    if connected:
        assert connected_components(A, directed=False)[0] == 1


def test_grid_structure():
    g = gen.grid(32, 24)
    assert g.n == 768 and g.m == 2 * (2 * 32 * 24 - 32 - 24)
    _check_csr(g)
    deg = np.diff(g.rowptr)
    assert deg.min() == 2 and deg.max() == 4
    gu = gen.grid(16, 10, "uniform", seed=3)
    assert gu.w.min() >= 0.5 and gu.w.max() < 1.5
    _check_csr(gu)
    # edge enumeration order: vertex 0's right edge gets the first draw
    u0 = gen.uniform01(3, 2)
    assert gu.w[gu.rowptr[0]] == 0.5 + u0[0]  # edge (0,1)
    assert gu.w[gu.rowptr[0] + 1] == 0.5 + u0[1]  # edge (0,10)


def test_grid_with_hub_structure():
    g = gen.grid_with_hub(16, 10, 4, seed=3)
    _check_csr(g)
    deg = np.diff(g.rowptr)
    hub = g.n - 1
    assert g.n == 161 and deg[hub] == 40
    assert np.array_equal(g.col[g.rowptr[hub]:], np.arange(0, 160, 4))
    assert np.all(g.w[g.rowptr[hub]:] == 1.0)
    # the grid part keeps the grid's edges and weights
    gu = gen.grid(16, 10, "uniform", seed=3)
    for v in (0, 5, 77, 159):
        row = dict(zip(g.col[g.rowptr[v]:g.rowptr[v + 1]], g.w[g.rowptr[v]:g.rowptr[v + 1]]))
        ref = dict(zip(gu.col[gu.rowptr[v]:gu.rowptr[v + 1]], gu.w[gu.rowptr[v]:gu.rowptr[v + 1]]))
        assert {k: x for k, x in row.items() if k != hub} == ref
        assert (hub in row) == (v % 4 == 0)


def test_grid_c2_sizes():
    g = gen.grid_1024x1000()
    assert g.n == 1024000 and g.m == 4091952


def test_rgg_brute_force_small():
    n, seed = 400, 9
    g = gen.rgg(n, seed, lcc=False)
    r = math.sqrt(8.0 / (math.pi * n))
    u = gen.uniform01(seed, 2 * n)
    x, y = u[0::2], u[1::2]
    G = int(1 / r)
    cell = np.minimum((y * G).astype(int), G - 1) * G + np.minimum((x * G).astype(int), G - 1)
    order = np.argsort(cell, kind="stable")
    px, py = x[order], y[order]
    d2 = (px[:, None] - px[None, :]) ** 2 + (py[:, None] - py[None, :]) ** 2
    adj = (d2 < r * r) & ~np.eye(n, dtype=bool)
    A = csr_matrix((g.w, g.col, g.rowptr), shape=(n, n)).toarray()
    assert np.array_equal(A > 0, adj)
    assert np.allclose(A[adj], np.exp(-d2[adj] / (r * r)), rtol=1e-15, atol=0)
    _check_csr(g, connected=False)


def test_rgg_lcc_connected():
    g = gen.rgg(20000, 5)
    _check_csr(g)
    assert g.n > 19900


def test_er_degree_and_connectivity():
    g = gen.erdos_renyi(5000, 6.0 / 4999, 3)
    _check_csr(g)
    assert abs(g.m / g.n - 6.0) < 0.3
    assert g.w.min() >= 0.5 and g.w.max() < 1.5


def test_random_connected_dyadic():
    g = gen.random_connected(40, 1, dyadic=True)
    _check_csr(g)
    assert np.all(g.w * 8 == np.round(g.w * 8))


@pytest.mark.parametrize("n", [200, 2000])
def test_batch_mix_members(n):
    gs = gen.batch_mix(count=6, seed=4, nmin=n, nmax=n + 10)
    for g in gs:
        _check_csr(g)


def _golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    with open(path) as f:
        return [int(t) for t in (l.strip() for l in f) if t and not t.startswith("#")]


def test_paper_square_grid_sizes():
    """The grid family of the paper's scaling table: every listed vertex count
    is a perfect square k*k, and the generator's k x k grid has exactly that
    many vertices and 2k(k-1) edges (checked on the smallest listed size)."""
    counts = _golden("table_4_2_square_grid_nodes.txt")
    assert len(counts) == 20 and counts == sorted(counts)
    ks = [math.isqrt(n) for n in counts]
    assert all(k * k == n for k, n in zip(ks, counts))
    k = ks[0]
    g = gen.grid(k, k)
    assert g.n == counts[0] == 326 * 326
    assert len(g.col) == 2 * (2 * k * (k - 1))  # both directions stored
