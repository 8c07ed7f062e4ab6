"""Candidate and final selection of the oracle on the hand-built cases in
tests/golden/select_cases.json (expected values derived by hand)."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "select_cases.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)


def test_select_cases(oracle_mod):
    for c in _cases()["select"]:
        out = oracle_mod.select(np.array(c["mw"]), np.array(c["m1"]), np.array(c["mk"], np.int32), c["sx"],
                                c["sy"], c["level"], c["min_score"], c["dmin"], c["max_out"])
        got = [list(r) for r in out.rows()]
        assert len(got) == len(c["expect"]), c["name"]
        for g, e in zip(got, c["expect"]):
            assert g[:3] == e[:3] and np.allclose(g[3:], e[3:]), c["name"]


def test_final_cases(oracle_mod):
    for c in _cases()["final"]:
        a = np.array(c["cands"], dtype=np.float64)
        cand = oracle_mod.Candidates(a[:, 0].astype(np.int32), a[:, 1].astype(np.int32), a[:, 2].astype(np.int32),
                                     a[:, 3], a[:, 4])
        out = oracle_mod.final(cand, c["min_score"], c["dmin"], c["max_out"])
        got = [list(r) for r in out.rows()]
        assert len(got) == len(c["expect"]), c["name"]
        for g, e in zip(got, c["expect"]):
            assert g[:3] == e[:3] and np.allclose(g[3:], e[3:]), c["name"]
