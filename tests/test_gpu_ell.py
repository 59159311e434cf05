"""The smoothing sweeps' ELL storage (slot-major blocks of the colours of
levels of more than 8,192 rows whose padding is cheap) against the CSR tile
sweeps and against the oracle.

The ELL sweep keeps the CSR sweep's rows per block, arithmetic and summation
order, so a hierarchy built with ELL blocks and one built without give
bitwise-equal solves: same schedule, same eigenvalue, same vector.  The 5-point
grids take four slots per row on level 0 and twelve on the coarse levels, the
8-neighbour (king's move) grids eight; the 1024 x 1000 grid's colours are
large enough for two rows per thread; the random geometric graph's level 0
(rows of up to 26 entries) keeps CSR for its large colours and takes 28-slot
blocks for its small dense ones.
"""
import numpy as np
import pytest

import gen
from test_gpu_parity import check_fp32_result

pytestmark = pytest.mark.gpu


def king(rows, cols, seed):
    """rows x cols grid with the 8 king's-move neighbours; weights U[0.5, 1.5]
    in the order right, down, down-right, down-left per vertex."""
    r, c = np.divmod(np.arange(rows * cols, dtype=np.int64), cols)
    v = r * cols + c
    nbr = [(c + 1 < cols, v + 1), (r + 1 < rows, v + cols),
           ((r + 1 < rows) & (c + 1 < cols), v + cols + 1),
           ((r + 1 < rows) & (c > 0), v + cols - 1)]
    a = np.stack([v] * 4, axis=1).reshape(-1)
    b = np.stack([t for _, t in nbr], axis=1).reshape(-1)
    keep = np.stack([k for k, _ in nbr], axis=1).reshape(-1)
    a, b = a[keep], b[keep]
    w = 0.5 + gen.uniform01(seed, a.shape[0])
    return gen._csr_from_undirected(rows * cols, a, b, w, f"king{rows}x{cols}")


CASES = {
    "grid320x300u": (lambda: gen.grid(320, 300, "uniform", seed=7), 4),
    "king300x300": (lambda: king(300, 300, 8), 8),
    "grid1024x1000": (lambda: gen.grid_1024x1000(), 4),
    "king1280x1280": (lambda: king(1280, 1280, 9), 8),
    "rgg200k": (lambda: gen.rgg(200000, 3), 28),
}
_graphs = {}


def graph(name):
    if name not in _graphs:
        _graphs[name] = CASES[name][0]()
    return _graphs[name]


# the grid parameters of the benchmark, at most 100 finest rounds
SOLVE = dict(seed=1, tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1,
             max_outer=100, tol_coarse=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_ell_sweeps_equal_csr_sweeps(fv, ctx, name, prec):
    g, ew = graph(name), CASES[name][1]
    print(f"case {name} {prec}", flush=True)
    he = fv.build_hierarchy_graph(ctx, g)
    hc = fv.build_hierarchy_graph(ctx, g, ell=False)
    # the ELL blocks: slots per row of each colour's block, 4 + 8 + 4 bytes a slot
    blocks = 0
    for lvl in range(he.levels - 1):
        rows = np.bincount(he.export_level(lvl).colour, minlength=he.colours[lvl])
        blocks += sum(16 * he.ell_width(lvl, c) * int(rows[c]) for c in range(he.colours[lvl]))
        assert all(hc.ell_width(lvl, c) == 0 for c in range(he.colours[lvl]))
    assert he.ell_width(0, he.colours[0] - 1) == ew
    assert he.device_bytes() - hc.device_bytes() >= blocks > 0
    re = fv.fiedler_solve(ctx, he, prec=prec, **SOLVE)
    rc = fv.fiedler_solve(ctx, hc, prec=prec, **SOLVE)
    assert re.schedule == rc.schedule
    assert re.lam == rc.lam and re.residual == rc.residual
    assert re.x.tobytes() == rc.x.tobytes()
    assert re.status == rc.status


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["grid320x300u", "king300x300", "rgg200k"])
def test_ell_replay_parity(fv, ctx, orc, name, prec):
    """The ELL path against the oracle on the oracle's schedule (the bars of the
    replay parity tests)."""
    g = graph(name)
    print(f"case {name} {prec} replay", flush=True)
    h = fv.build_hierarchy_graph(ctx, g)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
    ro = oh.solve(seed=1, omega=1.9)
    r = fv.fiedler_solve(ctx, h, prec=prec, seed=1, omega=1.9, replay=ro.counts)
    assert r.schedule == ro.counts
    if prec == "fp64":
        assert abs(r.lam - ro.lam) <= 1e-10 * abs(ro.lam)
        assert 1 - abs(float(r.x @ ro.x)) <= 1e-10
    else:
        check_fp32_result(g, r, ro, h.sigma[0])
