"""Pins of the oracle's 4-clique count (oracle.clique4, a generic join over the four
vertex variables; Section 3.1.3 runs the 4-clique query) against things it does not
compute itself: brute force over every combination of rows checked edge by edge,
closed forms on complete and transitive digraphs, and the binary hash-join plan with
closing-edge checks (pinned by tests/test_oracle_join.py)."""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import Query, Relation


def brute(q):
    """Every combination of eligible rows; a tuple counts when every edge holds."""
    sels = [oracle.eligible(r) for r in q.rels]
    cnt, chk = 0, 0
    for t in itertools.product(*[list(s) for s in sels]):
        if all(int(q.rels[a].cols[ca][t[a]]) == int(q.rels[b].cols[cb][t[b]]) for a, ca, b, cb in q.edges):
            cnt += 1
            f = 1
            for r, rid in enumerate(t):
                f = (f * int(oracle.lib().orc_chk_factor(r, int(rid)))) % (1 << 64)
            chk = (chk + f) % (1 << 64)
    return cnt, chk


def tiny(seed, rows=4, nv=3):
    rng = np.random.default_rng(seed)
    rels = [Relation(n, [rng.integers(0, nv, rows).astype(np.int32), rng.integers(0, nv, rows).astype(np.int32)])
            for n in ("AB", "AC", "AD", "BC", "BD", "CD")]
    return Query("k4", rels, list(W.CLIQUE4_EDGES), 0)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_tiny(seed):
    q = tiny(seed)
    assert oracle.clique4(q) == brute(q)


def test_brute_force_with_predicates_and_duplicates():
    pairs = np.array([(0, 0), (0, 1), (1, 0), (1, 1), (0, 0)], dtype=np.int32)   # (0, 0) twice
    rels = [Relation(n, [pairs[:, 0].copy(), pairs[:, 1].copy()]) for n in ("AB", "AC", "AD", "BC", "BD", "CD")]
    q = Query("k4", rels, list(W.CLIQUE4_EDGES), 0)
    full = brute(q)
    assert oracle.clique4(q) == full
    assert full[0] == sum(2 ** sum(1 for x, y in ((a, b), (a, c), (a, d), (b, c), (b, d), (c, d)) if x == y == 0)
                          for a in (0, 1) for b in (0, 1) for c in (0, 1) for d in (0, 1))
    q.rels[1].pred = (1, 1, 2)    # AC keeps c == 1
    q.rels[5].pred = (0, 0, 1)    # CD keeps c == 0: no tuple survives both
    assert oracle.clique4(q) == brute(q) == (0, 0)
    q.rels[5].pred = (1, 0, 1)    # CD keeps d == 0
    got = brute(q)
    assert oracle.clique4(q) == got and 0 < got[0] < full[0]


def complete(n, transitive):
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v and (u < v or not transitive)]
    src = np.array([p[0] for p in pairs], dtype=np.int32)
    dst = np.array([p[1] for p in pairs], dtype=np.int32)
    return src, dst


@pytest.mark.parametrize("n", [4, 5, 9, 13])
def test_closed_forms(n):
    # every ordered pair of distinct vertices: a, b, c, d all distinct, in any order
    assert oracle.clique4(W.clique4(*complete(n, False)))[0] == n * (n - 1) * (n - 2) * (n - 3)
    # u -> v iff u < v: a < b < c < d
    assert oracle.clique4(W.clique4(*complete(n, True)))[0] == math.comb(n, 4)


def test_parallel_rows_multiply():
    s, d = complete(6, True)
    q1 = W.clique4(s, d)
    q2 = W.clique4(np.concatenate([s, s]), np.concatenate([d, d]))
    assert oracle.clique4(q2)[0] == 64 * oracle.clique4(q1)[0]


@pytest.mark.parametrize("seed", range(4))
def test_equals_hash_join_on_small_power_law_graphs(seed):
    s, d = W.powerlaw_edges(600, 60, 2.3, 0xC11 + seed)
    q = W.clique4(s, d)
    tup, cnt, chk = oracle.hash_join(q)
    assert cnt > 0
    assert oracle.clique4(q) == (cnt, chk) == (tup.shape[0], oracle.checksum_of(tup))


def test_relabelled_query_same_result():
    """Another relation order, column order and root give the same tuples (permuted)."""
    s, d = W.powerlaw_edges(500, 50, 2.3, 0xC21)
    q = W.clique4(s, d)
    base = oracle.hash_join(q)[0]
    perm = [3, 5, 0, 2, 4, 1]                     # new position of each old relation
    inv = {old: new for new, old in enumerate(perm)}
    rels = [None] * 6
    for old, new in inv.items():
        R = q.rels[old]
        rels[new] = Relation(R.name, [R.cols[1], R.cols[0]])   # columns swapped
    edges = [(inv[a], 1 - ca, inv[b], 1 - cb) for a, ca, b, cb in q.edges]
    q2 = Query("k4b", rels, edges, root=4)
    tup2, cnt2, _ = oracle.hash_join(q2)
    assert cnt2 == base.shape[0]
    # the checksum uses relation positions: compare tuples mapped back to the old order
    back = np.empty_like(tup2)
    for old, new in inv.items():
        back[:, old] = tup2[:, new]
    assert oracle.clique4(q2) == (cnt2, oracle.checksum_of(tup2))
    assert np.array_equal(back[np.lexsort(back.T[::-1])], base[np.lexsort(base.T[::-1])])


def test_roles_reject_other_shapes():
    assert oracle.clique4_roles(W.config1(scale=0.001)) is None
    s, d = complete(5, True)
    assert oracle.clique4_roles(W.clique3(s, d)) is None
    q = W.clique4(s, d)
    q.edges = q.edges[:-1]                        # d no longer joins CD to AD
    assert oracle.clique4_roles(q) is None
    q = W.clique4(s, d)
    q.edges = q.edges + [(3, 0, 3, 1)]            # BC.src = BC.dst merges b and c
    assert oracle.clique4_roles(q) is None
    roles = oracle.clique4_roles(W.clique4(s, d))
    assert roles == [(0, 0, 1), (1, 0, 1), (2, 0, 1), (3, 0, 1), (4, 0, 1), (5, 0, 1)]


def test_stored_vote_network_value_recomputes():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "clique_wiki.json")) as fh:
        doc = json.load(fh)
    q = W.config6(k=4)
    assert q.rels[0].nrows == doc["edges"]
    assert oracle.clique4(q) == (doc["clique4"]["count"], doc["clique4"]["checksum"])
