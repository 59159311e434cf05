"""GPU parity at the benchmark sizes, in the benchmark's launch configuration.

* 1024 x 1000 grid (U[0.5,1.5] weights): the whole hierarchy bit-exact against
  the oracle; the FP32-mixed solve run exactly as the benchmark runs it reaches
  residual <= 1e-6, checked again on the CPU in FP64 from the returned vector;
  its eigenvalue is within 1e-5 of the FP64 oracle on the same schedule, and the
  FP64 GPU solve on that schedule within 1e-10.
* 4M-vertex random geometric graph: the whole hierarchy bit-exact; FP64 and
  FP32-mixed solves on a short replayed schedule against the oracle.
* Batch of graphs drawn from the 4096-graph benchmark mix (grids and
  Erdos-Renyi graphs with pendant vertices): one FP32-mixed batched launch;
  every item that reaches residual <= 1e-6 has its eigenvalue within 1e-5 of
  the FP64 oracle on the same schedule, and at least 20 of the 24 items do.
* The smallest square grid of the paper's scaling table (326 x 326, unit
  weights): FP32-mixed and FP64 solves with the square-grid parameters reach
  residual <= 1e-6 and their eigenvalues lie within the Kato-Temple bound
  r^2 / (2 lambda_2 - lambda) of lambda_2 = 2 - 2 cos(pi / 326).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen
from test_gpu_parity import compare_structure

pytestmark = pytest.mark.gpu

from bench import SOLVE as BENCH_SOLVE  # the benchmark's solve parameters
from bench import SQUARE_SOLVE  # the square-grid scaling workload's


def laplacian(g):
    W = sp.csr_matrix((g.w, g.col, g.rowptr), shape=(g.n, g.n))
    return sp.diags(np.asarray(W.sum(axis=1)).ravel()) - W


def cpu_residual(g, x, lam):
    r = laplacian(g) @ x - lam * x
    return float(np.linalg.norm(r) / np.linalg.norm(x))


def test_grid_1024x1000_benchmark_configuration(fv, ctx, orc):
    g = gen.grid_1024x1000()
    print("case grid1024x1000: structure", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=25)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
    compare_structure(h, oh)
    print("case grid1024x1000: fp32 solve as benchmarked", flush=True)
    r32 = fv.fiedler_solve(ctx, h, prec="fp32", **BENCH_SOLVE)
    assert r32.status == 0 and r32.residual <= 1e-6
    assert abs(float(r32.x @ r32.x) - 1.0) <= 1e-12 and abs(float(r32.x.sum())) <= 1e-9
    assert cpu_residual(g, r32.x, r32.lam) <= 1e-6 * (1 + 1e-6)
    ro = oh.solve(seed=1, omega=1.9, replay=r32.schedule)
    assert abs(r32.lam - ro.lam) <= 1e-5 * ro.lam
    print("case grid1024x1000: fp64 replay", flush=True)
    r64 = fv.fiedler_solve(ctx, h, prec="fp64", seed=1, omega=1.9, replay=r32.schedule)
    assert abs(r64.lam - ro.lam) <= 1e-10 * ro.lam
    assert 1.0 - abs(float(r64.x @ ro.x)) <= 1e-10
    assert abs(r64.residual - ro.residual) <= 1e-9 * ro.residual
    h.free()


def test_rgg_4m_structure_and_short_schedule(fv, ctx, orc):
    g = gen.rgg_4m()
    print(f"case rgg4m n={g.n}: structure", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=25)
    oh = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
    compare_structure(h, oh)
    J = h.levels - 1
    sched = [300] + [2, 1] * J
    print("case rgg4m: fp64 / fp32 replay", flush=True)
    ro = oh.solve(seed=1, omega=1.9, replay=sched)
    r64 = fv.fiedler_solve(ctx, h, prec="fp64", seed=1, omega=1.9, replay=sched)
    assert r64.schedule == ro.counts
    assert abs(r64.lam - ro.lam) <= 1e-10 * ro.lam
    assert 1.0 - abs(float(r64.x @ ro.x)) <= 1e-10
    r32 = fv.fiedler_solve(ctx, h, prec="fp32", seed=1, omega=1.9, replay=sched)
    assert abs(r32.lam - ro.lam) <= 1e-5 * ro.lam
    h.free()


def test_batch_mix_sample_against_oracle(fv, ctx, orc):
    graphs = gen.batch_mix(4096)
    pick = [int(v % 4096) for v in gen.splitmix64(11, 24)]
    sample = [graphs[i] for i in pick]
    print(f"case batch-mix sample of {len(sample)}: n={[g.n for g in sample]}", flush=True)
    hs = [fv.build_hierarchy_graph(ctx, g, n_coarse=25) for g in sample]
    solve = dict(BENCH_SOLVE, max_outer=200)
    res = fv.fiedler_solve_batch(ctx, hs, prec="fp32", **solve)
    converged = 0
    for g, h, r in zip(sample, hs, res):
        ro = orc.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25).solve(
            seed=1, omega=1.9, replay=r.schedule)
        if r.residual <= 1e-6:
            converged += 1
            assert abs(r.lam - ro.lam) <= 1e-5 * abs(ro.lam), g.name
            assert ro.residual <= 2e-6, g.name
        h.free()
    assert converged >= 20, converged


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_paper_square_grid_closed_form(fv, ctx, prec):
    k = 326
    g = gen.grid(k, k)
    print(f"case grid{k}x{k} {prec}", flush=True)
    h = fv.build_hierarchy_graph(ctx, g, n_coarse=25)
    r = fv.fiedler_solve(ctx, h, prec=prec, **SQUARE_SOLVE)
    lam2 = 2 - 2 * math.cos(math.pi / k)  # a double eigenvalue; the next one is 2 lam2
    assert r.residual <= 1e-6
    res_cpu = cpu_residual(g, r.x, r.lam)
    assert res_cpu <= 1.01e-6
    assert abs(r.lam - lam2) <= res_cpu ** 2 / (2 * lam2 - r.lam) * 1.01
