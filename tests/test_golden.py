"""Regression pin: the oracle still reproduces its stored plain-workload results."""
import json
import os

import numpy as np

from oracle import eri_cd as E, mo, selfenergy as SE
from paper_0912_1459_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "plain_oracle.json")


def test_oracle_matches_stored_plain_results():
    g = json.load(open(GOLD))
    w = I.make("plain")
    V = E.eri_matrix(w.centres, w.alpha)
    for d, m in g["nvec"].items():
        assert E.pivoted_cd(float(d), V=V).M == m
    r = E.pivoted_cd(g["delta"], V=V)
    assert [int(p) for p in r.piv] == g["pivots"]
    Bsel, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, w.targets)
    res = SE.solve_targets(Bsel, Bvo, w.eps, w.nocc, w.targets, conv=g["conv"])
    assert np.abs(np.array([x.omega for x in res]) - g["omega"]).max() < 1e-11
    assert np.abs(np.array([x.pole for x in res]) - g["pole"]).max() < 1e-9
    assert [x.status for x in res] == g["status"]
