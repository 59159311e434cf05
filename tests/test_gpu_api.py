"""GPU tests of the C ABI's edges: header errors, the Laplacian input form,
device outputs of the batch, and the serving loop's cold mode, eviction under an
HBM budget, full queue and unknown tickets."""
import time

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def _wait(srv, tickets, limit=120):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < limit:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.001)
    return out


@pytest.mark.parametrize("n", [0, 1])
def test_header_errors(fv, ctx, orc, n):
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(0, np.int32)
    w = np.zeros(0)
    assert orc.input_to_adjacency(n, rp, col, w, True)[0] == fv.E_INVALID
    with pytest.raises(fv.FiedlerError) as e:
        fv.build_hierarchy(ctx, n, rp, col, w, is_adjacency=True)
    assert e.value.status == fv.E_INVALID


def test_laplacian_form_diagonal_checked(fv, ctx, orc):
    g = gen.random_connected(40, 5)
    L = gen.adjacency_to_laplacian(g.n, g.rowptr, g.col, g.w)
    rp, col, val = L
    h = fv.build_hierarchy(ctx, g.n, rp, col, val, is_adjacency=False, n_coarse=8)
    ha = fv.build_hierarchy_graph(ctx, g, n_coarse=8)
    assert h.export_level(0).w.tobytes() == ha.export_level(0).w.tobytes()
    bad = val.copy()
    diag = [p for i in range(g.n) for p in range(rp[i], rp[i + 1]) if col[p] == i]
    bad[diag[3]] *= 1.0 + 1e-9  # diagonal no longer the weighted degree
    expect = orc.input_to_adjacency(g.n, rp, col, bad, False)[0]
    assert expect == fv.E_NOT_LAPLACIAN
    with pytest.raises(fv.FiedlerError) as e:
        fv.build_hierarchy(ctx, g.n, rp, col, bad, is_adjacency=False)
    assert e.value.status == expect


def test_batch_device_outputs_equal_host_outputs(fv, ctx):
    from paper_1602_04386_amd.devmem import DeviceArray

    gs = [gen.grid(40 + 3 * k, 30, "uniform", seed=k) for k in range(4)] + \
         [gen.erdos_renyi(800, 6 / 799, 40 + k) for k in range(3)]
    hs = [fv.build_hierarchy_graph(ctx, g, n_coarse=25) for g in gs]
    host = fv.fiedler_solve_batch(ctx, hs, prec="fp32", max_outer=20, tol_res=1e-6, omega=1.9,
                                  tol_cos=3e-12, max_gs=30, max_pi=1)
    xs = [DeviceArray(dtype=np.float64, count=g.n) for g in gs]
    dev = fv.fiedler_solve_batch(ctx, hs, x_out=xs, prec="fp32", max_outer=20, tol_res=1e-6,
                                 omega=1.9, tol_cos=3e-12, max_gs=30, max_pi=1)
    for a, b, x in zip(host, dev, xs):
        assert a.lam == b.lam and a.schedule == b.schedule
        assert np.array_equal(a.x, x.numpy())


def test_server_cold_mode_and_budget_eviction(fv, ctx):
    gs = [gen.grid(30 + 4 * k, 24, "uniform", seed=20 + k) for k in range(4)]
    kw = dict(prec="fp32", tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1,
              max_outer=50)
    ref = fv.fiedler_solve_batch(ctx, [fv.build_hierarchy_graph(ctx, g, n_coarse=8) for g in gs],
                                 **kw)
    # cold: no cache, every request builds and frees its hierarchy
    srv = fv.Server(ctx, max_inflight=4, cache_hierarchies=False, n_coarse=8, **kw)
    tk = [srv.submit(k, g) for k, g in enumerate(gs)]
    out = _wait(srv, tk)
    srv.close()
    assert len(out) == len(tk)
    for k, t in enumerate(tk):
        assert not out[t][0]["cache_hit"]
        assert np.array_equal(out[t][1], ref[k].x)
    # cached under a budget that holds about one hierarchy: later requests
    # evict earlier ones and still get the same results
    ctx2 = fv.Context(0)
    h1 = fv.build_hierarchy_graph(ctx2, gs[-1], n_coarse=8)
    budget = int(h1.device_bytes() * 2.5)
    h1.free()
    srv = fv.Server(ctx2, max_inflight=1, hbm_budget_bytes=budget, n_coarse=8, **kw)
    order = [0, 1, 2, 3, 0, 1]
    tk = [srv.submit(k, gs[k]) for k in order]
    out = _wait(srv, tk)
    srv.close()
    ctx2.close()
    assert len(out) == len(tk)
    for k, t in zip(order, tk):
        assert out[t][0]["status"] == 0
        assert np.array_equal(out[t][1], ref[k].x)


def _drain(srv, tickets, limit=120):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < limit:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.0005)
    return out


def test_server_small_requests_do_not_wait_for_large_ones(fv, ctx):
    """A large request (the 1024 x 1000 grid) submitted first and small ones
    right after it: the small ones are admitted by the small-request lane
    while the large solve runs, and each result is published when its own
    work ends, so every small request completes before the large one; every
    result is bitwise the same as in the warm-up round, where the requests
    were admitted in other combinations."""
    kw = dict(prec="fp32", tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1,
              max_outer=50)
    big = gen.grid_1024x1000()
    small = [gen.grid(20 + k, 15, "uniform", seed=k) for k in range(6)]
    srv = fv.Server(ctx, max_inflight=8, n_coarse=25, **kw)
    # warm-up: every hierarchy cached, so the timed round has no builds
    warm = [srv.submit(100, big)] + [srv.submit(k, g) for k, g in enumerate(small)]
    first = _drain(srv, warm)
    assert len(first) == len(warm)
    print("case server lanes: timed round", flush=True)
    tickets = [srv.submit(100, big)] + [srv.submit(k, g) for k, g in enumerate(small)]
    out = _drain(srv, tickets)
    srv.close()
    assert len(out) == len(tickets)
    lat_big = out[tickets[0]][0]["latency_ms"]
    lat_small = [out[t][0]["latency_ms"] for t in tickets[1:]]
    assert max(lat_small) < lat_big, (lat_small, lat_big)
    for a, b in zip(warm, tickets):
        assert np.array_equal(first[a][1], out[b][1])
        assert first[a][0]["lambda"] == out[b][0]["lambda"]


def test_server_busy_and_unknown_ticket(fv, ctx):
    big = gen.grid(200, 150, "uniform", seed=3)
    srv = fv.Server(ctx, max_inflight=1, queue_capacity=1, n_coarse=25, prec="fp32",
                    max_outer=5)
    t1 = srv.submit(1, big)
    busy = 0
    tickets = [t1]
    for k in range(2):
        try:
            tickets.append(srv.submit(2 + k, big))
        except fv.FiedlerError as e:
            assert e.status == fv.E_BUSY
            busy += 1
    assert busy >= 1
    out = _wait(srv, tickets)
    assert len(out) == len(tickets)
    with pytest.raises(fv.FiedlerError) as e:
        srv.poll(987654321)
    assert e.value.status == fv.E_UNKNOWN_TICKET
    srv.close()


def test_server_tight_budget_many_workers_finishes(fv):
    """Four workers under a budget of about 1.5 hierarchies: workers that hold
    hierarchies while others need memory must not wait on each other forever.
    Every request ends with a status; the successful ones equal the batch
    results, the others report E_BUDGET."""
    print("server tight budget, 4 workers", flush=True)
    gs = [gen.grid(60 + 6 * k, 50, "uniform", seed=40 + k) for k in range(6)]
    kw = dict(prec="fp32", tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1,
              max_outer=50)
    ref_ctx = fv.Context(0)
    hs = [fv.build_hierarchy_graph(ref_ctx, g, n_coarse=8) for g in gs]
    hbytes = max(h.device_bytes() for h in hs)
    ref = fv.fiedler_solve_batch(ref_ctx, hs, **kw)
    ref_ctx.close()
    ctx = fv.Context(0)
    srv = fv.Server(ctx, max_inflight=4, hbm_budget_bytes=int(hbytes * 1.5), n_coarse=8, **kw)
    order = [k % len(gs) for k in range(24)]
    tk = [srv.submit(k, gs[k]) for k in order]
    out = _wait(srv, tk, limit=100)
    srv.close()
    ctx.close()
    assert len(out) == len(tk), f"{len(tk) - len(out)} requests never finished"
    ok = 0
    for k, t in zip(order, tk):
        st = out[t][0]["status"]
        assert st in (fv.OK, fv.E_BUDGET), st
        if st == fv.OK:
            ok += 1
            assert np.array_equal(out[t][1], ref[k].x)
    assert ok >= 1


def test_process_exit_with_objects_left_open(fv):
    """A program that ends with a context, a hierarchy, a server and device
    arrays still open exits cleanly: the binding's exit handlers release them
    while the HIP runtime still works (a hipFree from a finaliser after the
    runtime's own teardown aborted the process with std::bad_variant_access)."""
    import os
    import subprocess
    import sys
    import textwrap

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {root!r})
        import numpy as np
        import gen
        import paper_1602_04386_amd as fv
        from paper_1602_04386_amd.devmem import DeviceArray
        ctx = fv.Context(0)
        g = gen.grid(64, 48, "uniform", seed=7)
        h = fv.build_hierarchy_graph(ctx, g, n_coarse=8)
        x = DeviceArray(dtype=np.float64, count=g.n)
        r = fv.fiedler_solve(ctx, h, x_out=x, prec="fp32", max_outer=5, tol_res=1e-6)
        y = DeviceArray(np.arange(10.0))
        srv = fv.Server(ctx, max_inflight=2, n_coarse=8, prec="fp32", max_outer=3)
        t = srv.submit(1, g)
        print("left open", r.lam, flush=True)
    """)
    print("exit-with-open-objects subprocess", flush=True)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, (p.returncode, p.stdout[-2000:], p.stderr[-2000:])
    assert "left open" in p.stdout
