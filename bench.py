"""Benchmark: Fiedler solves per second on one MI355X, with the roofline of the
level-0 smoothing kernel and the CPU oracle timed beside it.

Workload: 1024 x 1000 5-point grid (n = 1,024,000, 4,091,952 stored
off-diagonals), edge weights iid U[0.5, 1.5] from SplitMix64 seed 2, input
CSR resident in HBM.  One step = the whole path: device setup (matching,
aggregation, Galerkin, colouring) plus the cascadic solve to a finest-level
residual ||L x - lambda x|| / ||x|| <= 1e-6, in FP32-mixed precision.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# SOR factor 1.9, per-phase cosine tolerance 3e-12, at most 40 sweeps and one
# power step per phase, finest rounds repeated until the residual is <= 1e-6.
SOLVE = dict(seed=1, tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=40, max_pi=1,
             max_outer=400, max_coarsest=100000)
N_COARSE = 25


def pass_bytes(n, m, prec):
    """Algorithmic bytes of one smoothing sweep / power step over a level: the
    matrix read once (index + value), row pointers, x read once, x written."""
    return (8 * m + 4 * (n + 1) + 8 * n) if prec == "fp32" else (12 * m + 4 * (n + 1) + 16 * n)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--roofline-sweeps", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np

    import gen
    import paper_1602_04386_amd as fv
    from paper_1602_04386_amd.devmem import DeviceArray, hip

    g = gen.grid_1024x1000()
    ctx = fv.Context(0)
    # Input CSR and output resident in HBM before any timed work.
    rp, col, w = DeviceArray(g.rowptr), DeviceArray(g.col), DeviceArray(g.w)
    x = DeviceArray(dtype=np.float64, count=g.n)
    hip().hipDeviceSynchronize()

    def step():
        h = fv.build_hierarchy(ctx, g.n, rp, col, w, is_adjacency=True, n_coarse=N_COARSE)
        r = fv.fiedler_solve(ctx, h, x_out=x, prec=args.prec, **SOLVE)
        return h, r

    for _ in range(args.warmup):
        h, r = step()
        h.free()
    log(f"warmup done: residual {r.residual:.3e}")
    lat, res, lams, sched = [], [], [], None
    hip().hipDeviceSynchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        h, r = step()
        lat.append((time.perf_counter() - ts) * 1e3)
        res.append(r.residual)
        lams.append(r.lam)
        sched = r.schedule
        levels = (h.n, h.nnz, h.colours)
        h.free()
    hip().hipDeviceSynchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    ok = all(v <= SOLVE["tol_res"] for v in res)

    # Setup and solve split (one more step, timed separately).
    ts = time.perf_counter()
    h = fv.build_hierarchy(ctx, g.n, rp, col, w, is_adjacency=True, n_coarse=N_COARSE)
    t_setup = (time.perf_counter() - ts) * 1e3
    ts = time.perf_counter()
    r = fv.fiedler_solve(ctx, h, x_out=x, prec=args.prec, **SOLVE)
    t_solve = (time.perf_counter() - ts) * 1e3

    # Roofline of the level-0 smoothing kernel: two replayed schedules that
    # differ only in the number of level-0 sweeps; the device-time difference
    # divided by the sweep count is one sweep (ncolours launches).
    J = h.levels - 1
    S0, S1 = 2, 2 + args.roofline_sweeps

    def sweep_sched(s):
        return [0] + [0, 0] * (J - 1) + [s, 0]

    def dev_ms(s):
        best = float("inf")
        for _ in range(3):
            rr = fv.fiedler_solve(ctx, h, x_out=x, prec=args.prec, seed=1,
                                  replay=sweep_sched(s))
            best = min(best, rr.t_solve_ms)
        return best

    t_a, t_b = dev_ms(S0), dev_ms(S1)
    log(f"roofline replays: {S0} sweeps {t_a:.3f} ms, {S1} sweeps {t_b:.3f} ms")
    t_sweep_ms = (t_b - t_a) / (S1 - S0)
    n0, m0, c0 = h.n[0], h.nnz[0], h.colours[0]
    bytes_sweep = pass_bytes(n0, m0, args.prec)
    achieved = bytes_sweep / (t_sweep_ms * 1e-3) / 1e9
    h.free()

    # The same solve in the other precision, on the same hierarchy build, for
    # the FP32-mixed versus FP64 comparison (eigenvalue difference, solves/s).
    other = "fp64" if args.prec == "fp32" else "fp32"
    t_o, r_o = [], None
    for _ in range(2):
        ts = time.perf_counter()
        h = fv.build_hierarchy(ctx, g.n, rp, col, w, is_adjacency=True, n_coarse=N_COARSE)
        r_o = fv.fiedler_solve(ctx, h, x_out=x, prec=other, **SOLVE)
        t_o.append(time.perf_counter() - ts)
        h.free()
    log(f"{other} leg: {min(t_o) * 1e3:.1f} ms, residual {r_o.residual:.3e}")

    out = {
        "metric": "Fiedler solves/s at residual<=1e-6 (grid 1024x1000, setup+solve)",
        "value": round(args.steps / elapsed, 4) if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "p50_ms": round(statistics.median(lat), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32-mixed" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "grid 1024x1000, weights iid U[0.5,1.5] (SplitMix64 seed 2), "
                        "n=1024000, nnz=4091952",
            "n_coarse": N_COARSE, "solve": SOLVE, "levels": len(levels[0]),
            "level_n": levels[0], "level_colours": levels[2],
            "residual_max": max(res), "lambda": lams[-1], "converged": ok,
            "setup_ms": round(t_setup, 3), "solve_ms": round(t_solve, 3),
            "schedule_head": sched[:12] if sched else None,
            "finest_rounds": (len(sched) - 1 - 2 * J) // 2 if sched else None,
        },
        "roofline": {
            "kernel": "k_gs_tile<float> (level 0)" if args.prec == "fp32"
                      else "k_gs_tile<double> (level 0)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_sweep": bytes_sweep,
            "launches_per_sweep": c0,
            "avg_launch_us": round(t_sweep_ms * 1e3 / c0, 3),
            "sweep_us": round(t_sweep_ms * 1e3, 3),
        },
    }
    out["other_precision"] = {
        "dtype": "f64" if other == "fp64" else "fp32-mixed",
        "value": round(1.0 / min(t_o), 4) if r_o.residual <= SOLVE["tol_res"] else 0.0,
        "unit": "solves/s", "residual": r_o.residual, "lambda": r_o.lam,
        "lambda_rel_diff": abs(r_o.lam - lams[-1]) / abs(r_o.lam),
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(g, args.prec)
    print(json.dumps(out))


def cpu_baseline(g, prec):
    """The FP64 oracle, one thread, on one full setup + solve of the same
    grid with the same solve parameters (a bounded sample)."""
    import oracle

    oracle.build()
    t = time.perf_counter()
    h = oracle.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=N_COARSE)
    t_setup = time.perf_counter() - t
    r = h.solve(**SOLVE)
    total = time.perf_counter() - t
    return {"value": round(1.0 / total, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one setup+solve of the same grid, FP64, same parameters "
                      f"(setup {t_setup:.1f} s, total {total:.1f} s, residual {r.residual:.2e})"}


if __name__ == "__main__":
    main()
