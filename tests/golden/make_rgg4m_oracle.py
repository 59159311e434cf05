"""Writes the FP64 oracle's solves of the 4M-point random geometric graph
(SplitMix64 seed 3): its schedule, eigenvalue and residual, and the entries of
its vector at 4096 positions drawn with SplitMix64 seed 12.

* rgg4m_oracle.json: SOR factor 1.9, cosine tolerance 3e-12, at most 30 sweeps
  and one power step per phase, at most 20 finest rounds (the 1024 x 1000
  grid's parameters; this graph stalls above residual 1e-6 under them).
* rgg4m_oracle_own.json: the random geometric graph's own parameters: no
  cosine stop, 30 sweeps and 30 power steps per phase, finest rounds until
  residual 1e-6 (at most 100).

Calls only the oracle; each takes a few minutes on one core.
Run: python tests/golden/make_rgg4m_oracle.py [short|own]
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
OWN = dict(SOLVE, tol_cos=0.0, max_gs=30, max_pi=30, max_outer=100)
RECORDS = {"short": ("rgg4m_oracle.json", SOLVE), "own": ("rgg4m_oracle_own.json", OWN)}


def main(which):
    oracle.build()
    g = gen.rgg_4m()
    h = oracle.Hierarchy(g.n, g.rowptr, g.col, g.w, n_coarse=25)
    idx = sorted(set(int(v % g.n) for v in gen.splitmix64(12, 4096)))
    for key in which:
        name, params = RECORDS[key]
        r = h.solve(**params)
        out = {"graph": "rgg_4m(seed=3)", "n": g.n, "nnz": int(len(g.col)), "solve": params,
               "status": int(r.status), "schedule": [int(v) for v in r.counts],
               "lambda": r.lam, "residual": r.residual, "sample_index": idx,
               "sample_x": [float(r.x[i]) for i in idx], "xmax": float(abs(r.x).max())}
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(out, f)
        print(name, "lambda", r.lam, "residual", r.residual, "schedule length", len(r.counts))


if __name__ == "__main__":
    main(sys.argv[1:] or list(RECORDS))
