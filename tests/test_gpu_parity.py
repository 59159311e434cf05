"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.

Bars:
* integer and structural results (matching, aggregates, colouring, coarse
  graphs, shifts) are bit-exact, coarse weights included;
* FP64: lambda within 1e-10 relative and 1 - |cos(x_gpu, x_oracle)| <= 1e-10
  when the GPU runs the oracle's schedule (replay);
* FP32-mixed: lambda within 1e-5 relative of the FP64 oracle, the vector within
  1 - |cos| <= 1e-8 of the oracle's iterate on the same schedule, and the
  reported eigenvalue and residual those of the returned vector recomputed on
  the CPU in FP64 (see check_fp32_result);
* free-running schedules equal the oracle's on these inputs.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen

pytestmark = pytest.mark.gpu


def cpu_rq_residual(g, x):
    """Rayleigh quotient x^T L x / x^T x and residual ||L x - rho x|| / ||x|| of
    x on the input graph, in FP64 with plain sparse algebra (Definition 2.1:
    L = D - W with D the weighted degrees)."""
    W = sp.csr_matrix((g.w, g.col, g.rowptr), shape=(g.n, g.n))
    d = np.asarray(W.sum(axis=1)).ravel()
    Lx = d * x - W @ x
    rho = float(x @ Lx) / float(x @ x)
    return rho, float(np.linalg.norm(Lx - rho * x) / np.linalg.norm(x))


def check_fp32_result(g, r, ro, sigma0):
    """An FP32-mixed GPU result r against the FP64 oracle result ro of the same
    schedule.

    FP32 storage rounds every stored entry to 2^-24 relative; over the few
    hundred sweeps of a schedule the iterates drift apart by at most the sum
    of those roundings in the modes the iteration does not damp, which leaves
    1 - |cos| far below 1e-8 (a vector difference of 1.4e-4).  The eigenvalue
    and residual the library reports must be those of the vector it returns:
    recomputed on the CPU in FP64 they agree to 1e-9 relative (summation order
    only).  Finally the residual map x -> ||(L - rho(x)) x|| is 4 sigma-Lipschitz
    on unit vectors (||L|| <= sigma), which bounds the residual gap by the
    vector gap."""
    # distance between the unit vectors up to sign: 1 - |cos| = dist^2 / 2,
    # computed from the difference (1 - |cos| itself underflows to 0)
    s = 1.0 if float(r.x @ ro.x) >= 0 else -1.0
    dist = float(np.linalg.norm(r.x - s * ro.x))
    assert dist * dist / 2 <= 1e-8, dist
    rho, res = cpu_rq_residual(g, r.x)
    assert abs(rho - r.lam) <= 1e-9 * abs(r.lam) + 1e-15, (rho, r.lam)
    assert abs(res - r.residual) <= 1e-9 * res + 1e-14, (res, r.residual)
    assert abs(res - ro.residual) <= 4 * sigma0 * dist + 1e-12, (res, ro.residual, dist)
    assert abs(r.lam - ro.lam) <= 1e-5 * abs(ro.lam)

CASES = {
    "c1_grid32x24": (lambda: gen.grid_32x24(), 8),
    "path64": (lambda: gen.path(64), 8),
    "path2": (lambda: gen.path(2), 8),
    "rand200": (lambda: gen.random_connected(200, 7), 8),
    "grid64x48u": (lambda: gen.grid(64, 48, "uniform", seed=3), 25),
    "er3000": (lambda: gen.erdos_renyi(3000, 6 / 2999, 11), 25),
    "rgg20k": (lambda: gen.rgg(20000, 5), 25),
    "grid256x250u": (lambda: gen.grid(256, 250, "uniform", seed=2), 25),
    # a 3,200-entry row on a multi-workgroup level (longer than a tile's
    # staging capacity: the row takes the direct path) beside short rows
    "gridhub128x100": (lambda: gen.grid_with_hub(128, 100, 4, seed=6), 25),
    # level 1 (4,173 rows) fits the engine's LDS with its column indices and
    # row pointers but not its FP32 weights: the engine reads only those from
    # global memory
    "grid96x96u": (lambda: gen.grid(96, 96, "uniform", seed=9), 25),
    # coarse levels of Erdos-Renyi graphs grow dense (levels of about 1,000
    # vertices and below average 30 to 120 neighbours): the one-workgroup
    # matching and colouring scan such rows with a whole wavefront
    "er12000": (lambda: gen.erdos_renyi(12000, 6 / 11999, 21), 25),
    # mean degree ~20: the row copies of levels 0 and 1 (20,000 and 9,683
    # rows) take groups of 16 lanes per row, and most of level 1's rows hold
    # more than 32 Galerkin terms
    "rgg20k_deg20": (lambda: gen.rgg(20000, 12, radius=math.sqrt(20 / (math.pi * 20000))), 25),
}
_graphs = {}


def graph(name):
    if name not in _graphs:
        f, nc = CASES[name]
        _graphs[name] = (f(), nc)
    return _graphs[name]


def compare_structure(h, oh):
    assert h.levels == oh.nlevels
    for l in range(h.levels):
        a, b = h.export_level(l), oh.level(l)
        assert (a.n, a.m) == (b.n, b.m), l
        assert np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.col, b.col), l
        assert a.w.tobytes() == b.w.tobytes(), l
        assert a.sigma == b.sigma, l
        if l + 1 < h.levels:
            assert np.array_equal(a.q, b.q), l
            assert np.array_equal(a.colour, b.colour) and a.ncolours == b.ncolours, l


@pytest.mark.parametrize("name", list(CASES))
def test_structure_bit_exact(fv, ctx, orc, name):
    g, nc = graph(name)
    print(f"case {name} n={g.n}", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    compare_structure(h, oh)


def test_concurrent_builds_bit_exact(fv, ctx, orc):
    """fv_build_hierarchies: every case built on four concurrent host threads
    and streams is the oracle's hierarchy bit for bit, and a graph with an
    isolated vertex among them fails alone with the oracle's status."""
    names = list(CASES)
    graphs = [graph(nm)[0] for nm in names]
    bad = gen._csr_from_undirected(5, np.array([0, 1, 2]), np.array([1, 2, 3]), np.ones(3))
    print(f"case concurrent builds of {len(graphs)} graphs and one invalid", flush=True)
    hs, st = fv.build_hierarchies(ctx, graphs[:3] + [bad] + graphs[3:], threads=4, n_coarse=25)
    assert st[3] == fv.E_ISOLATED and hs[3] is None
    del hs[3], st[3]
    assert st == [0] * len(graphs)
    for nm, g, h in zip(names, graphs, hs):
        nc = graph(nm)[1]
        if nc != 25:
            h.free()
            h = fv.build_hierarchies(ctx, [g], threads=1, n_coarse=nc)[0][0]
        compare_structure(h, orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc))
        h.free()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_replay_parity(fv, ctx, orc, name, prec):
    g, nc = graph(name)
    print(f"case {name} {prec}", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    ro = oh.solve(seed=1)
    r = fv.fiedler_solve(ctx, h, prec=prec, seed=1, replay=ro.counts)
    assert r.schedule == ro.counts
    rel = abs(r.lam - ro.lam) / abs(ro.lam)
    if prec == "fp64":
        assert rel <= 1e-10
        assert 1 - abs(float(r.x @ ro.x)) <= 1e-10
        assert abs(r.residual - ro.residual) <= 1e-9 * max(ro.residual, 1e-12) + 1e-14
    else:
        assert rel <= 1e-5
        check_fp32_result(g, r, ro, h.sigma[0])
    assert abs(np.linalg.norm(r.x) - 1) < 1e-12 and abs(r.x.sum()) < 1e-9 * math.sqrt(g.n)


@pytest.mark.parametrize("name", ["c1_grid32x24", "grid64x48u", "rgg20k", "grid256x250u"])
def test_free_run_schedule(fv, ctx, orc, name):
    g, nc = graph(name)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    ro = oh.solve(seed=1)
    r = fv.fiedler_solve(ctx, h, prec="fp64", seed=1)
    assert r.schedule == ro.counts
    assert abs(r.lam - ro.lam) <= 1e-10 * ro.lam


@pytest.mark.parametrize("name", ["c1_grid32x24", "grid64x48u", "rgg20k"])
def test_free_run_schedule_loose_coarsest(fv, ctx, orc, name):
    """A loose coarsest tolerance: the same first-crossing stop on both sides."""
    g, nc = graph(name)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    ro = oh.solve(seed=1, tol_coarse=1e-6)
    r = fv.fiedler_solve(ctx, h, prec="fp64", seed=1, tol_coarse=1e-6)
    assert r.schedule == ro.counts
    assert ro.counts[0] < oh.solve(seed=1).counts[0]
    assert abs(r.lam - ro.lam) <= 1e-10 * ro.lam


DEGENERATE = {
    "no_smoothing": dict(max_gs=0, max_pi=5, tol_res=0.0),
    "no_power_steps": dict(max_gs=20, max_pi=0, tol_res=0.0),
    "no_finest_rounds": dict(max_gs=20, max_pi=1, tol_res=1e-6, max_outer=0),
    "plain_gauss_seidel_rounds": dict(omega=1.0, max_gs=10, max_pi=1, tol_res=1e-3,
                                      max_outer=30),
    "single_sweep_cap": dict(omega=1.9, max_gs=1, max_pi=1, tol_res=1e-4, max_outer=40),
    # met by the cascade alone: the round enqueued ahead of the residual is void
    "tolerance_met_before_rounds": dict(max_gs=20, max_pi=1, tol_res=1.0, max_outer=50),
}


@pytest.mark.parametrize("name", ["c1_grid32x24", "grid256x250u"])
@pytest.mark.parametrize("params", list(DEGENERATE))
def test_degenerate_phase_limits(fv, ctx, orc, name, params):
    """Phase caps of zero and one, no finest rounds, and the plain sweep: the
    free-running GPU schedule equals the oracle's, one-workgroup engine
    (32x24) and multi-workgroup passes (256x250) alike."""
    g, nc = graph(name)
    kw = dict(seed=1, tol_cos=1e-8, **DEGENERATE[params])
    print(f"case {name} {params}", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    ro = oh.solve(**kw)
    r = fv.fiedler_solve(ctx, h, prec="fp64", **kw)
    assert r.status == ro.status  # E_NOT_CONVERGED on both when the rounds run out
    assert r.schedule == ro.counts
    assert abs(r.lam - ro.lam) <= 1e-10 * abs(ro.lam)


def test_c1_closed_form_tight(fv, ctx):
    """32x24 unit grid: lambda_2 = 2 - 2 cos(pi/32) (the small FP64 workload)."""
    g = gen.grid_32x24()
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=8)
    r = fv.fiedler_solve(ctx, h, prec="fp64", tol_cos=1e-10, tol_res=1e-9, max_gs=2000,
                         max_pi=50, max_outer=5000)
    lam = 2 - 2 * math.cos(math.pi / 32)
    assert r.status == 0 and r.residual <= 1e-9
    assert abs(r.lam - lam) <= 1e-10 * lam
    phi = np.repeat(np.cos(math.pi * (np.arange(32) + 0.5) / 32), 24)
    phi /= np.linalg.norm(phi)
    assert 1 - abs(float(r.x @ phi)) <= 1e-8


def test_tol_res_loop_matches_oracle(fv, ctx, orc):
    g, nc = graph("grid64x48u")
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    kw = dict(seed=1, tol_cos=1e-12, tol_res=1e-6, max_gs=2000, max_pi=2, max_outer=400,
              omega=1.8)
    ro = oh.solve(**kw)
    r = fv.fiedler_solve(ctx, h, prec="fp64", replay=ro.counts, **kw)
    assert r.residual <= 1.01e-6 and ro.residual <= 1e-6
    assert abs(r.lam - ro.lam) <= 1e-10 * ro.lam
    rf = fv.fiedler_solve(ctx, h, prec="fp32", **kw)
    assert abs(rf.lam - ro.lam) <= 1e-5 * ro.lam
    # both stop at residual <= 1e-6 (free-running): the FP32 result's own
    # residual, recomputed on the CPU, meets the tolerance
    assert cpu_rq_residual(g, rf.x)[1] <= 1.01e-6
    rr = fv.fiedler_solve(ctx, h, prec="fp32", replay=ro.counts, **kw)
    check_fp32_result(g, rr, ro, h.sigma[0])


def test_sor_relaxation_replay(fv, ctx, orc):
    g, nc = graph("grid64x48u")
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    ro = oh.solve(seed=1, omega=1.7, tol_cos=1e-10, max_gs=300)
    r = fv.fiedler_solve(ctx, h, prec="fp64", seed=1, omega=1.7, replay=ro.counts)
    assert abs(r.lam - ro.lam) <= 1e-10 * ro.lam


def test_laplacian_and_device_inputs(fv, ctx):
    from paper_1602_04386_amd.devmem import DeviceArray

    g = gen.grid(40, 33, "uniform", seed=8)
    h1 = fv.build_hierarchy_graph(ctx, g, n_coarse=10)
    rp, col, val = g.laplacian()
    h2 = fv.build_hierarchy(ctx, g.n, rp, col, val, is_adjacency=False, n_coarse=10)
    h3 = fv.build_hierarchy(ctx, g.n, DeviceArray(g.rowptr), DeviceArray(g.col),
                            DeviceArray(g.w), is_adjacency=True, n_coarse=10)
    for h in (h2, h3):
        assert h.levels == h1.levels
        for l in range(h.levels):
            a, b = h.export_level(l), h1.export_level(l)
            assert np.array_equal(a.col, b.col) and a.w.tobytes() == b.w.tobytes()
    r1 = fv.fiedler_solve(ctx, h1)
    xd = DeviceArray(dtype=np.float64, count=g.n)
    fv.fiedler_solve(ctx, h3, x_out=xd)
    assert np.array_equal(r1.x, xd.numpy())


def test_repeatable_bitwise(fv, ctx):
    g, nc = graph("grid256x250u")
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    a = fv.fiedler_solve(ctx, h, prec="fp32")
    b = fv.fiedler_solve(ctx, h, prec="fp32")
    assert np.array_equal(a.x, b.x) and a.lam == b.lam and a.schedule == b.schedule


def _bad_inputs():
    g = gen.random_connected(12, 3)
    rp, col, w = g.rowptr.copy(), g.col.copy(), g.w.copy()
    w2 = w.copy()
    w2[0] += 1e-3
    w3 = w.copy()
    w3[1] = -w3[1]
    c2 = col.copy()
    c2[rp[0]], c2[rp[0] + 1] = c2[rp[0] + 1], c2[rp[0]]
    c3 = col.copy()
    c3[-1] = g.n
    return [
        ("asym", g.n, rp, col, w2, True),
        ("negative", g.n, rp, col, w3, True),
        ("unsorted", g.n, rp, c2, w, True),
        ("col_range", g.n, rp, c3, w, True),
        ("isolated", 3, np.array([0, 1, 2, 2], np.int32), np.array([1, 0], np.int32),
         np.array([1.0, 1.0]), True),
    ]


@pytest.mark.parametrize("case", _bad_inputs(), ids=lambda c: c[0])
def test_input_errors_match_oracle(fv, ctx, orc, case):
    name, n, rp, col, w, adj = case
    expect = orc.input_to_adjacency(n, rp, col, w, adj)[0]
    with pytest.raises(fv.FiedlerError) as e:
        fv.build_hierarchy(ctx, n, rp, col, w, is_adjacency=adj)
    assert e.value.status == expect


def test_degenerate_graphs(fv, ctx, orc):
    # star: every leaf joins the centre's aggregate -> one level, big coarsest
    k = 100
    a = np.zeros(k, np.int64)
    b = np.arange(1, k + 1)
    g = gen._csr_from_undirected(k + 1, a, b, np.ones(k))
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=8)
    assert h.levels == 1
    r = fv.fiedler_solve(ctx, h)
    assert abs(r.lam - 1.0) < 1e-9 and r.residual < 1e-9
    # two components (no isolated vertex): lambda_2 = 0
    a = np.array([0, 2])
    b = np.array([1, 3])
    g2 = gen._csr_from_undirected(4, a, b, np.ones(2))
    h2 = fv.build_hierarchy_graph(ctx, g2, n_coarse=8)
    r2 = fv.fiedler_solve(ctx, h2)
    assert abs(r2.lam) < 1e-12


def test_batch_matches_oracle_and_is_mix_independent(fv, ctx, orc):
    gs = [gen.grid(30 + k, 20, "uniform", seed=k) for k in range(3)] + \
         [gen.random_connected(300, 50 + k) for k in range(3)] + [gen.path(64), gen.grid_32x24()]
    hs = [fv.build_hierarchy_graph(ctx, g, n_coarse=8) for g in gs]
    res = fv.fiedler_solve_batch(ctx, hs, prec="fp64")
    for g, r in zip(gs, res):
        ro = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=8).solve(seed=1)
        assert r.schedule == ro.counts
        assert abs(r.lam - ro.lam) <= 1e-10 * ro.lam
        assert 1 - abs(float(r.x @ ro.x)) <= 1e-10
    alone = fv.fiedler_solve_batch(ctx, [hs[4]], prec="fp64")[0]
    assert np.array_equal(alone.x, res[4].x) and alone.lam == res[4].lam


def test_server_results_equal_batch(fv, ctx, orc):
    import time

    gs = [gen.grid(20 + k, 15, "uniform", seed=k) for k in range(6)]
    srv = fv.Server(ctx, max_inflight=4, n_coarse=8, prec="fp32")
    tickets = [srv.submit(k, g) for k, g in enumerate(gs)]
    tickets += [srv.submit(0, gs[0])]  # second request for a cached graph
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < 60:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.001)
    srv.close()
    assert len(out) == len(tickets)
    hs = [fv.build_hierarchy_graph(ctx, g, n_coarse=8) for g in gs]
    ref = fv.fiedler_solve_batch(ctx, hs, prec="fp32")
    for k, t in enumerate(tickets):
        info, x = out[t]
        gi = k if k < len(gs) else 0
        assert info["status"] == 0
        assert np.array_equal(x, ref[gi].x)
    assert out[tickets[-1]][0]["cache_hit"]
    # served results against the oracle: the FP64 oracle run on the schedule
    # the served (= batched) solve took
    for gi in (0, 3, 5):
        g = gs[gi]
        info, x = out[tickets[gi]]
        ro = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=8).solve(
            seed=1, replay=ref[gi].schedule)
        served = ref[gi]
        assert served.lam == info["lambda"] and np.array_equal(served.x, x)
        check_fp32_result(g, served, ro, hs[gi].sigma[0])


def test_server_large_requests_take_the_single_graph_path(fv, ctx):
    # a finest level above the batched launch's limit runs through the
    # multi-workgroup path on the worker's own workspace: same bits as the
    # single-graph call, also while small requests run beside it
    import time

    big = gen.grid(160, 120, "uniform", seed=9)  # 19,200 vertices
    small = [gen.grid(20 + k, 15, "uniform", seed=k) for k in range(3)]
    kw = dict(prec="fp32", tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1,
              max_outer=50)
    srv = fv.Server(ctx, max_inflight=8, n_coarse=25, **kw)
    tickets = [srv.submit(100, big)] + [srv.submit(k, g) for k, g in enumerate(small)]
    tickets.append(srv.submit(100, big))  # cached hierarchy, second run
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < 120:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.001)
    srv.close()
    assert len(out) == len(tickets)
    h = fv.build_hierarchy_graph(ctx, big, n_coarse=25)
    ref = fv.fiedler_solve(ctx, h, **kw)
    for t in (tickets[0], tickets[-1]):
        info, x = out[t]
        assert info["status"] == ref.status
        assert np.array_equal(x, ref.x) and info["lambda"] == ref.lam


# Long phases without the cosine stop and many power steps per phase (the
# random geometric graph's and the serving pool's parameters): every phase
# runs to its cap, so the schedule is fixed by the parameters alone and the
# GPU's free-running schedule must be the oracle's.
LONG_PHASES = dict(seed=1, tol_cos=0.0, max_gs=30, max_pi=30, omega=1.95, tol_res=1e-6,
                   max_outer=6, tol_coarse=1e-6)


@pytest.mark.parametrize("name", ["grid64x48u", "er3000", "rgg20k", "grid256x250u"])
def test_long_phase_parameters(fv, ctx, orc, name):
    g, nc = graph(name)
    print(f"case {name} long phases", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=nc)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=nc)
    ro = oh.solve(**LONG_PHASES)
    # single-graph path (multi-workgroup passes on the large levels), FP64
    r = fv.fiedler_solve(ctx, h, prec="fp64", **LONG_PHASES)
    assert r.schedule == ro.counts
    assert abs(r.lam - ro.lam) <= 1e-10 * ro.lam
    assert 1 - abs(float(r.x @ ro.x)) <= 1e-10
    # the batched engine on the same graph, FP64 and FP32-mixed
    rb = fv.fiedler_solve_batch(ctx, [h], prec="fp64", **LONG_PHASES)[0]
    assert rb.schedule == ro.counts
    assert abs(rb.lam - ro.lam) <= 1e-10 * ro.lam
    r32 = fv.fiedler_solve(ctx, h, prec="fp32", **LONG_PHASES)
    check_fp32_result(g, r32, oh.solve(**dict(LONG_PHASES, replay=r32.schedule)), h.sigma[0])


# The serving policy's early exit (fv_solve_opts.early_exit): the finest rounds
# end once the residual cannot reach tol_res in the rounds left at its last
# reduction factor.  Two random geometric graphs that stall (one solved in the
# engine, one with its finest level on the multi-workgroup passes) and one
# that converges within the cap.
EARLY_CASES = {
    "rgg1.5k": (1523, gen.derive_seed(5, 22) ^ 0x55),
    "rgg10k": (10381, gen.derive_seed(5, 10) ^ 0x55),
    "rgg3k": (3000, 11),
}
SERVE_PHASES = dict(LONG_PHASES, max_outer=12)


@pytest.mark.parametrize("name", list(EARLY_CASES))
def test_early_exit_matches_oracle(fv, ctx, orc, name):
    n, seed = EARLY_CASES[name]
    g = gen.rgg(n, seed)
    print(f"case {name} early exit", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=25)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
    ro = oh.solve(early_exit=True, **SERVE_PHASES)
    # FP64: the oracle's schedule, its rounds included, and its result
    r = fv.fiedler_solve(ctx, h, prec="fp64", early_exit=True, **SERVE_PHASES)
    assert r.schedule == ro.counts
    assert r.status == ro.status
    assert abs(r.residual - ro.residual) <= 1e-9 * ro.residual
    assert abs(r.lam - ro.lam) <= 1e-10 * ro.lam
    rb = fv.fiedler_solve_batch(ctx, [h], prec="fp64", early_exit=True, **SERVE_PHASES)[0]
    assert rb.schedule == ro.counts and rb.status == ro.status
    # FP32-mixed: the same rule on its own residuals; a stalling graph stops
    # well before the cap, a converging one runs as without early exit
    r32 = fv.fiedler_solve(ctx, h, prec="fp32", early_exit=True, **SERVE_PHASES)
    r32_full = fv.fiedler_solve(ctx, h, prec="fp32", **SERVE_PHASES)
    J = h.levels - 1
    rounds = (len(r32.schedule) - 1 - 2 * J) // 2
    if ro.status == 0:
        assert r32.schedule == r32_full.schedule and r32.residual == r32_full.residual
    else:
        assert rounds < SERVE_PHASES["max_outer"] and r32.status == fv.E_NOT_CONVERGED


def test_server_early_exit_results_equal_batch(fv, ctx):
    """Served requests under the early exit (small random geometric graphs,
    stalling and converging, mixed in one admission) give the batched
    launch's results bit for bit: the same schedules, statuses and vectors."""
    import time

    gs = [gen.rgg(n, seed) for n, seed in EARLY_CASES.values() if n <= 4000]
    gs += [gen.rgg(2500, 31), gen.rgg(1800, 32)]
    srv = fv.Server(ctx, max_inflight=4, n_coarse=25, prec="fp32", early_exit=True,
                    **{k: v for k, v in SERVE_PHASES.items() if k != "seed"})
    tickets = [srv.submit(k, g) for k, g in enumerate(gs)]
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < 60:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.001)
    srv.close()
    assert len(out) == len(tickets)
    hs = [fv.build_hierarchy_graph(ctx, g, n_coarse=25) for g in gs]
    ref = fv.fiedler_solve_batch(ctx, hs, prec="fp32", early_exit=True, **SERVE_PHASES)
    statuses = set()
    for k, t in enumerate(tickets):
        info, x = out[t]
        assert info["status"] == ref[k].status and info["lambda"] == ref[k].lam
        assert np.array_equal(x, ref[k].x)
        statuses.add(ref[k].status)
    assert statuses == {0, fv.E_NOT_CONVERGED}  # both kinds are in the mix
