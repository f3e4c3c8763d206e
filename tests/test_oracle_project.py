"""Pins of oracle.project (value tuples of a join result, Section 2.2's result as
values rather than row ids), against properties that hold for any correct projection:

* every value tuple satisfies the query's equalities on the projected join columns
  (a value taken from the wrong relation or the wrong row breaks one);
* a column holding each row's own index projects back to the row ids exactly;
* the sorted multiset of value tuples equals the one a nested-loop join over the
  relations' values produces directly, without row ids.
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W


def value_join_brute(q, cols):
    """Nested loops over rows of every relation, emitting the chosen values of each
    combination that satisfies all edges and predicates."""
    out = []
    ranges = [range(r.nrows) for r in q.rels]
    for rows in itertools.product(*ranges):
        ok = True
        for i, rel in enumerate(q.rels):
            if rel.pred is not None and not (rel.pred[1] <= int(rel.cols[rel.pred[0]][rows[i]]) < rel.pred[2]):
                ok = False
                break
        if not ok:
            continue
        if all(int(q.rels[a].cols[ca][rows[a]]) == int(q.rels[b].cols[cb][rows[b]]) for a, ca, b, cb in q.edges):
            out.append(tuple(int(q.rels[r].cols[c][rows[r]]) for r, c in cols))
    return sorted(out)


@pytest.mark.parametrize("seed", range(60))
def test_projection_satisfies_the_join_and_equals_a_value_join(seed):
    q = W.tiny_random(3000 + seed)
    if np.prod([max(1, r.nrows) for r in q.rels]) > 200_000:
        pytest.skip("cross product too large for the value brute force")
    tup, cnt, _ = oracle.hash_join(q)
    cols = oracle.default_projection(q)
    vals = oracle.project(q, tup)
    assert vals.shape == (cnt, len(cols))
    where = {rc: i for i, rc in enumerate(cols)}
    for a, ca, b, cb in q.edges:
        assert np.array_equal(vals[:, where[(a, ca)]], vals[:, where[(b, cb)]])
    assert sorted(map(tuple, vals.tolist())) == value_join_brute(q, cols)


def test_identity_column_projects_to_row_ids():
    rng = np.random.default_rng(4)
    rels = []
    for i, n in enumerate([30, 40, 25]):
        key_a = rng.integers(0, 6, n).astype(np.int32)
        key_b = rng.integers(0, 6, n).astype(np.int32)
        ident = np.arange(n, dtype=np.int32)
        rels.append(W.Relation("R%d" % i, [key_a, key_b, ident], None))
    q = W.Query("ident", rels, [(0, 1, 1, 0), (1, 1, 2, 0)], 0)
    tup, cnt, _ = oracle.hash_join(q)
    assert cnt > 0
    got = oracle.project(q, tup, [(2, 2), (0, 2), (1, 2)])
    assert np.array_equal(got[:, 0], tup[:, 2].astype(np.int32))
    assert np.array_equal(got[:, 1], tup[:, 0].astype(np.int32))
    assert np.array_equal(got[:, 2], tup[:, 1].astype(np.int32))
