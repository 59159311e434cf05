"""Spectral partitioning (recursive bisection of the Fiedler vector) against
the oracle's counterpart.

* Exact: the oracle's recursion, given the library's own Fiedler vector of
  each subgraph it extracts (solved through the C ABI), must produce the same
  labels bit for bit: this checks the subgraph extraction, the median and
  sign cuts with their tie rule, the isolated-vertex rule and the relabelling.
* Whole method: against the oracle's recursion with the oracle's own FP64
  solves, the labels agree (the vectors agree to ~1e-10 and the gaps between
  neighbouring values at the cut are far larger) and the cut weight matches.
* Balance: median cuts give parts whose sizes differ by at most the vertices
  that were isolated in their part.
"""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

KW = dict(prec="fp64", seed=1, tol_cos=1e-10, max_gs=200, max_pi=10)

CASES = {
    "grid64x48u": lambda: gen.grid(64, 48, "uniform", seed=31),
    "rgg8000": lambda: gen.rgg(8000, 32),
    "er3000": lambda: gen.erdos_renyi(3000, 6 / 2999, 33),  # pendant vertices
}


def cut_weight(g, labels):
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    m = (labels[rows] != labels[g.col]) & (g.col > rows)
    return float(g.w[m].sum())


@pytest.mark.parametrize("cut", ["median", "sign"])
@pytest.mark.parametrize("name", list(CASES))
def test_partition_matches_oracle_recursion(fv, ctx, orc, name, cut):
    g = CASES[name]()
    parts = 8
    print(f"partition {name} {cut} parts={parts}", flush=True)
    labels, st = fv.spectral_partition(ctx, g, parts=parts, cut=cut, **KW)

    def gpu_vector(sub):
        h = fv.build_hierarchy(ctx, sub.n, sub.rowptr, sub.col, sub.w, True)
        r = fv.fiedler_solve(ctx, h, **KW)
        h.free()
        return r.x

    ref, n_iso = orc.spectral_partition(g, parts, cut, vector=gpu_vector)
    assert np.array_equal(labels, ref)
    assert st["parts"] == parts and st["solves"] == parts - 1
    sizes = np.bincount(labels, minlength=parts)
    assert sizes.min() == st["part_size_min"] and sizes.max() == st["part_size_max"]
    assert abs(st["cut_weight"] - cut_weight(g, labels)) <= 1e-9 * max(1.0, st["cut_weight"])
    assert abs(st["total_weight"] - g.w.sum() / 2) <= 1e-9 * g.w.sum()
    if cut == "median":
        assert sizes.max() - sizes.min() <= 1 + n_iso
    if name == "er3000" and cut == "median":
        assert n_iso > 0  # the isolated-vertex rule was exercised


@pytest.mark.parametrize("name", ["grid64x48u", "rgg8000"])
def test_partition_against_oracle_solves(fv, ctx, orc, name):
    g = CASES[name]()
    labels, st = fv.spectral_partition(ctx, g, parts=4, cut="median", **KW)
    ref, _ = orc.spectral_partition(g, 4, "median", **{k: v for k, v in KW.items() if k != "prec"})
    assert np.mean(labels != ref) <= 1e-3
    assert abs(cut_weight(g, ref) - st["cut_weight"]) <= 1e-2 * cut_weight(g, ref)


def test_partition_errors(fv, ctx):
    g = gen.grid(10, 8)
    for parts in (1, 3, 6):
        with pytest.raises(fv.FiedlerError) as e:
            fv.spectral_partition(ctx, g, parts=parts)
        assert e.value.status == fv.E_INVALID
