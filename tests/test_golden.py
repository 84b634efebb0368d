"""Regression fixtures written by tests/golden/make_golden.py (oracle only)."""
import json
import os

import pytest

from tests.golden.make_golden import CASES, digest, run

FIX = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_fixtures.json")))


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_matches_fixture(name):
    e = FIX[name]
    r = run(CASES[name])
    assert r["nnzL"] == e["nnzL"] and r["P"] == e["P"] and r["D"] == e["D"]
    for k in ("perm", "parent", "colcount", "gmap", "node_of", "node_begin", "node_size"):
        assert digest(r[k]) == e[k + "_sha256"], k
