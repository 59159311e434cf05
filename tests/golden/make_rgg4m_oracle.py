"""Writes tests/golden/rgg4m_oracle.json: the FP64 oracle's solve of the
4M-point random geometric graph (SplitMix64 seed 3) with the benchmark's
parameters for that graph (SOR factor 1.9, cosine tolerance 3e-12, at most 30
sweeps and one power step per phase, at most 20 finest rounds) -- its schedule,
eigenvalue and residual, and the entries of its vector at 4096 positions drawn
with SplitMix64 seed 12.  Calls only the oracle; takes a few minutes on one
core.  Run: python tests/golden/make_rgg4m_oracle.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

SOLVE = dict(seed=1, tol_cos=3e-12, tol_res=1e-6, omega=1.9, max_gs=30, max_pi=1, max_outer=20,
             max_coarsest=100000, tol_coarse=1e-6)


def main():
    oracle.build()
    g = gen.rgg_4m()
    h = oracle.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
    r = h.solve(**SOLVE)
    idx = sorted(set(int(v % g.n) for v in gen.splitmix64(12, 4096)))
    out = {"graph": "rgg_4m(seed=3)", "n": g.n, "nnz": int(len(g.col)), "solve": SOLVE,
           "status": int(r.status), "schedule": [int(v) for v in r.counts],
           "lambda": r.lam, "residual": r.residual, "sample_index": idx,
           "sample_x": [float(r.x[i]) for i in idx], "xmax": float(abs(r.x).max())}
    with open(os.path.join(HERE, "rgg4m_oracle.json"), "w") as f:
        json.dump(out, f)
    print("lambda", r.lam, "residual", r.residual, "schedule length", len(r.counts))


if __name__ == "__main__":
    main()
