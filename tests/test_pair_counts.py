"""Connected-pair counts: the oracle's whole-space counter is pinned to
closed forms and to the per-row scan; the plan's single and double pair
counts (the terms behind the benchmark's terms/s) equal the oracle's exact
counts, stored in tests/golden/pair_counts.json by
tests/golden/make_pair_counts.py (oracle only)."""
import json
import os
from math import comb

import numpy as np
import pytest

from paper_2501_18185_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _fci_counts(n, na, nb):
    """Ordered pairs of an FCI space by excitation level: every determinant
    has the same neighbours (singles: one electron of one spin moves;
    doubles: two of one spin, or one of each)."""
    ndet = comb(n, na) * comb(n, nb)
    s = na * (n - na) + nb * (n - nb)
    d = comb(na, 2) * comb(n - na, 2) + comb(nb, 2) * comb(n - nb, 2) + na * (n - na) * nb * (n - nb)
    return ndet * s, ndet * d


def test_oracle_pair_counts_fci_closed_form(orc):
    for n, na, nb in [(8, 4, 4), (10, 3, 3), (9, 4, 2)]:
        p = synth.Problem("spinfree", n, na, nb, synth.space_fci(n, na, nb), np.zeros((n, n)), np.zeros((n,) * 4), 0.0)
        assert orc.pair_counts(p) == _fci_counts(n, na, nb)


def test_oracle_pair_counts_equal_row_scan(orc):
    """On random selected spaces (spin-free and spinor) the counter equals the
    sum of the per-row degrees of the oracle's excitation analysis."""
    rng = np.random.default_rng(3)
    d = synth.space_selected_spinfree(12, 4, 4, 3000, rng)
    p = synth.Problem("spinfree", 12, 4, 4, d, np.zeros((12, 12)), np.zeros((12,) * 4), 0.0)
    s, dd = orc.pair_counts(p)
    assert s + dd == int(orc.degree_rows(p).sum())
    ds = synth.space_selected_spinor(8, 6, 2000, rng)
    q = synth.Problem("spinor", 8, 6, -1, ds, np.zeros((16, 16)), np.zeros((16,) * 4), 0.0)
    s, dd = orc.pair_counts(q)
    assert s + dd == int(orc.degree_rows(q).sum())


def _golden():
    path = os.path.join(HERE, "golden", "pair_counts.json")
    if not os.path.exists(path):
        pytest.fail("tests/golden/pair_counts.json missing: run tests/golden/make_pair_counts.py")
    with open(path) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("name", ["sci-n64-10a10b-2e6", "spinor-40kp-20e-1e6", "batch16-problem0",
                                  "batch16-problem7", "batch16-problem15"])
def test_plan_pair_counts_equal_oracle(name):
    """Host plan (no GPU) of the benchmarked spaces: single and double pair
    counts equal the oracle's exact whole-space counts."""
    from paper_2501_18185_amd import mw
    g = _golden()[name]
    p = synth.workload(g["workload"], g["problem"])
    assert p.ndet == g["ndet"]
    pl = mw.Plan(p, upload=False)
    assert pl.info("single_pairs") == g["single_pairs"]
    assert pl.info("double_pairs") == g["double_pairs"]
    assert pl.info("pairs") == g["single_pairs"] + g["double_pairs"]
