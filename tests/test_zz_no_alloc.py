"""The allocation-free solve (fv_fiedler_solve_noalloc) against fv_fiedler_solve.

Both run the same kernels on the same hierarchy; the allocation-free one takes
its workspace from the library's fixed device scratch.  Results must be
bitwise equal (vector, eigenvalue, residual, schedule).  Two calls in a row,
the second on a smaller graph, show that the scratch left by the first call
does not leak into the second.  A context whose HBM budget leaves no room for
fv_fiedler_solve's workspace shows that the allocation-free solve needs none.
"""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a.status == b.status
    assert a.x.tobytes() == b.x.tobytes()
    assert a.lam == b.lam and a.residual == b.residual
    assert a.schedule == b.schedule


SOLVE = dict(seed=1, tol_cos=1e-8, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1, max_outer=60,
             tol_coarse=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_solve_two_calls(fv, prec):
    print(f"noalloc two calls prec={prec}", flush=True)
    ctx = fv.Context(0)
    big = gen.grid(300, 260, weights="uniform", seed=21)   # multi-workgroup levels + engine
    small = gen.grid(40, 31, weights="uniform", seed=22)   # engine only
    hb = fv.build_hierarchy_graph(ctx, big)
    hs = fv.build_hierarchy_graph(ctx, small)
    for h in (hb, hs):
        ref = fv.fiedler_solve(ctx, h, prec=prec, **SOLVE)
        got = fv.fiedler_solve_noalloc(ctx, h, prec=prec, **SOLVE)
        _same(got, ref)
    # once more on the big graph after the small one
    ref = fv.fiedler_solve(ctx, hb, prec=prec, **SOLVE)
    got = fv.fiedler_solve_noalloc(ctx, hb, prec=prec, **SOLVE)
    _same(got, ref)
    ctx.close()


def test_noalloc_replay_and_device_output(fv):
    """Replayed schedule and a device output buffer, as fv_fiedler_solve."""
    from paper_1602_04386_amd.devmem import DeviceArray

    print("noalloc replay + device output", flush=True)
    ctx = fv.Context(0)
    g = gen.grid(128, 97, weights="uniform", seed=23)
    h = fv.build_hierarchy_graph(ctx, g)
    ref = fv.fiedler_solve(ctx, h, prec="fp64", seed=3, tol_cos=1e-7)
    dx = DeviceArray(dtype=np.float64, count=g.n)
    got = fv.fiedler_solve_noalloc(ctx, h, x_out=dx, prec="fp64", seed=3, replay=ref.schedule)
    assert dx.numpy().tobytes() == ref.x.tobytes()
    assert got.lam == ref.lam and got.schedule == ref.schedule
    dx.free()
    ctx.close()


def test_noalloc_needs_no_budget(fv):
    """Under a budget that only fits the hierarchy, fv_fiedler_solve fails for
    want of workspace; the allocation-free solve runs."""
    print("noalloc under a tight budget", flush=True)
    g = gen.grid(200, 150, weights="uniform", seed=24)
    probe = fv.Context(0)
    hp = fv.build_hierarchy_graph(probe, g)
    hbytes = hp.device_bytes()
    ref = fv.fiedler_solve(probe, hp, prec="fp32", **SOLVE)
    probe.close()
    ctx = fv.Context(0, hbm_budget_bytes=hbytes + 4096)
    h = fv.build_hierarchy_graph(ctx, g)
    with pytest.raises(fv.FiedlerError) as e:
        fv.fiedler_solve(ctx, h, prec="fp32", **SOLVE)
    assert e.value.status == fv.E_BUDGET
    got = fv.fiedler_solve_noalloc(ctx, h, prec="fp32", **SOLVE)
    _same(got, ref)
    ctx.close()


def test_noalloc_rejects_oversized_graph(fv):
    """A level-0 graph whose workspace exceeds the fixed scratch is refused
    before anything runs."""
    print("noalloc oversized graph", flush=True)
    ctx = fv.Context(0)
    g = gen.grid(1200, 1200, weights="unit")  # 1.44M vertices: 3 x 8 B x n > 32 MiB
    h = fv.build_hierarchy_graph(ctx, g)
    with pytest.raises(fv.FiedlerError) as e:
        fv.fiedler_solve_noalloc(ctx, h, prec="fp32", **SOLVE)
    assert e.value.status == fv.E_SCRATCH
    # a graph that fits still runs afterwards
    g2 = gen.grid(64, 50, weights="uniform", seed=25)
    h2 = fv.build_hierarchy_graph(ctx, g2)
    _same(fv.fiedler_solve_noalloc(ctx, h2, prec="fp32", **SOLVE),
          fv.fiedler_solve(ctx, h2, prec="fp32", **SOLVE))
    ctx.close()
