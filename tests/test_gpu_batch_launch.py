"""The batched launch's configurations: the autotuner's choice, forced LDS
sizes and a captured-and-replayed hipGraph all give bitwise the results of the
default launch (the engine's arithmetic does not depend on where a level sits
or which workgroup takes a graph)."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

KW = dict(prec="fp32", tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1, max_outer=60,
          tol_coarse=1e-6)


def _mix():
    gs = []
    for k in range(12):
        n = int(300 * 1.45 ** k)
        if k % 2:
            a = max(4, int(round((4 * n / 3) ** 0.5)))
            gs.append(gen.grid(a, max(3, n // a), "uniform", seed=60 + k))
        else:
            gs.append(gen.erdos_renyi(n, 6.0 / (n - 1), 70 + k))
    return gs


def _same(a, b):
    for ra, rb in zip(a, b):
        assert ra.x.tobytes() == rb.x.tobytes()
        assert ra.lam == rb.lam and ra.schedule == rb.schedule and ra.status == rb.status


def test_configurations_bitwise_equal(fv):
    print("batch launch configurations", flush=True)
    ctx = fv.Context(0)
    gs = _mix()
    hs = [fv.build_hierarchy_graph(ctx, g) for g in gs]
    ref = fv.fiedler_solve_batch(ctx, hs, **KW)
    for lds in (32 << 10, 96 << 10, 144 << 10):
        info = {"lds_bytes": lds}
        _same(fv.fiedler_solve_batch(ctx, hs, batch=info, **KW), ref)
        assert info["lds_bytes_used"] == lds and not info["tuned"]
    info = {"autotune": 1}
    _same(fv.fiedler_solve_batch(ctx, hs, batch=info, **KW), ref)
    assert info["tuned"]
    again = {"autotune": 2}
    _same(fv.fiedler_solve_batch(ctx, hs, batch=again, **KW), ref)
    assert again["tuned"] and again["lds_bytes_used"] == info["lds_bytes_used"]
    ctx.close()


def test_captured_graph_replays(fv):
    print("batch launch graph capture", flush=True)
    ctx = fv.Context(0)
    gs = _mix()
    hs = [fv.build_hierarchy_graph(ctx, g) for g in gs]
    ref = fv.fiedler_solve_batch(ctx, hs, **KW)
    first = {"graph": 1}
    _same(fv.fiedler_solve_batch(ctx, hs, batch=first, **KW), ref)
    assert not first["replayed"]
    for _ in range(3):  # replays, with eager work between them
        info = {"graph": 1}
        _same(fv.fiedler_solve_batch(ctx, hs, batch=info, **KW), ref)
        assert info["replayed"]
        fv.fiedler_solve(ctx, hs[0], **KW)
    # a changed batch is captured anew, not replayed
    info = {"graph": 1}
    _same(fv.fiedler_solve_batch(ctx, hs[:5], batch=info, **KW), ref[:5])
    assert not info["replayed"]
    # a hierarchy rebuilt in place of a freed one never matches the old graph
    info = {"graph": 1}
    fv.fiedler_solve_batch(ctx, hs[:5], batch=info, **KW)
    assert info["replayed"]
    hs[4].free()
    hs[4] = fv.build_hierarchy_graph(ctx, gs[4])
    info = {"graph": 1}
    _same(fv.fiedler_solve_batch(ctx, hs[:5], batch=info, **KW), ref[:5])
    assert not info["replayed"]
    ctx.close()
