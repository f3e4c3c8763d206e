"""The stored oracle values of the serving mix (tests/golden/serving_mix.json) are
reproducible: every entry's draw gives the stored kind and sizes, and for the smallest
queries the oracle's join-tree DP and its binary hash join both recompute the stored
count and checksum."""
import json
import os

import pytest

import oracle
from workloads import serving as S

PATH = os.path.join(os.path.dirname(__file__), "golden", "serving_mix.json")


@pytest.fixture(scope="module")
def doc():
    with open(PATH) as fh:
        return json.load(fh)


def test_every_entry_matches_its_draw(doc):
    assert doc["n"] == len(doc["queries"]) == 256
    for e in doc["queries"]:
        sp = S.draw_spec(doc["seed"], e["index"], e["draw"], min_rows=doc["min_rows"], max_rows=doc["max_rows"])
        assert (sp.kind, list(sp.rows)) == (e["kind"], list(e["rows"])), e["index"]
        assert abs(sp.s - e["s"]) < 1e-12
        assert 0 <= e["count"] <= doc["count_cap"]


def test_smallest_entries_recompute(doc):
    for e in sorted(doc["queries"], key=lambda e: sum(e["rows"]))[:6]:
        sp = S.draw_spec(doc["seed"], e["index"], e["draw"], min_rows=doc["min_rows"], max_rows=doc["max_rows"])
        q = S.query_cpu(sp)
        assert oracle.join_tree_dp(q) == (e["count"], e["checksum"]), e["index"]
        _, cnt, chk = oracle.hash_join(q)
        assert (cnt, chk) == (e["count"], e["checksum"]), e["index"]
