"""Pins of the update-maintenance oracle (Section 2.4): counting filters and the
propagation of inserted tuples toward the root.

Counting filters are checked against the plain blocked filter (oracle.bf_build, the
C implementation): the support of the counters after inserting keys is exactly the
filter built from those keys; inserting A and B then deleting B leaves the counters of
A alone; a saturated counter survives deletions. Propagation is checked against what
it must preserve: the relation's own filter equals a rebuild from its grown rows, an
ancestor's filter is a subset of a rebuild's bits (only truly new keys are followed),
and every key that truly joins in the grown query is contained (no false negatives),
found by the binary hash join of the grown query.
"""
import numpy as np
import pytest

import oracle
import workloads as W

K, B = 6, 512
SEED32 = oracle.filter_seed(7)


def empty_counts(nb):
    return np.zeros((nb, B), dtype=np.uint8)


@pytest.mark.parametrize("n,nb", [(300, 8), (2000, 40), (50, 1)])
def test_counting_support_is_the_plain_filter(n, nb):
    keys = np.random.default_rng(n).integers(-2**31, 2**31, size=n).astype(np.int32)
    c = oracle.cf_update(empty_counts(nb), keys, +1, nb, K, B, SEED32)
    assert np.array_equal(oracle.cf_export(c), oracle.bf_build(keys, None, nb, K, B, SEED32))
    # every counter counts the pattern positions that land on it
    assert int(c.sum()) == n * K or c.max() == 15


def test_delete_undoes_insert_without_saturation():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 1 << 20, size=400).astype(np.int32)
    b = rng.integers(0, 1 << 20, size=300).astype(np.int32)
    nb = 64
    ca = oracle.cf_update(empty_counts(nb), a, +1, nb, K, B, SEED32)
    cab = oracle.cf_update(ca, b, +1, nb, K, B, SEED32)
    assert cab.max() < 15
    back = oracle.cf_update(cab, b, -1, nb, K, B, SEED32)
    assert np.array_equal(back, ca)
    assert np.array_equal(oracle.cf_export(back), oracle.bf_build(a, None, nb, K, B, SEED32))
    gone = oracle.cf_update(back, a, -1, nb, K, B, SEED32)
    assert not gone.any()


def test_saturated_counters_survive_deletions():
    nb = 4
    x = np.full(20, 12345, dtype=np.int32)
    c = oracle.cf_update(empty_counts(nb), x, +1, nb, K, B, SEED32)
    blk, pos = oracle.bf_pattern(12345, nb, K, B, SEED32)
    assert all(c[blk, p] == 15 for p in pos)
    c2 = oracle.cf_update(c, x, -1, nb, K, B, SEED32)
    assert np.array_equal(c2, c)
    words = oracle.cf_export(c2)
    assert oracle.bf_probe(words, x[:1], None, nb, K, B, SEED32).all()
    # removing a key that was never inserted changes nothing at zero counters
    z = oracle.cf_update(empty_counts(nb), np.array([7], dtype=np.int32), -1, nb, K, B, SEED32)
    assert not z.any()


def grown(q, rel, new_cols):
    rels = [W.Relation(r.name, [np.concatenate([c, nc]) if i == rel else c for c, nc in
                                zip(r.cols, new_cols if i == rel else r.cols)], r.pred)
            for i, r in enumerate(q.rels)]
    return W.Query(q.name + "+", rels, q.edges, q.root)


def backward_filters(q, bpk=4):
    _, F = oracle.sieve(q, bits_per_key=bpk, k=K, block_bits=B, passes=1, seed=7, root=q.root)
    return {j: F[("bwd", j)] for (kind, j) in F if kind == "bwd"}


@pytest.mark.parametrize("seed", range(12))
def test_propagation_preserves_what_it_must(seed):
    rng = np.random.default_rng(seed)
    kind = ["chain", "star"][seed % 2]
    if kind == "chain":
        q = W.chain(4, [300, 250, 200, 150], 60, 0.5, 0x5EED0C00 + seed)
    else:
        q = W.star(400, 3, 80, 0.5, 0x5EED0C00 + seed)
    rel = len(q.rels) - 1 if kind == "chain" else 1 + seed % 3
    F = backward_filters(q)
    t = oracle.JoinTree(len(q.rels), q.edges, q.root)
    nnew = 40
    new_cols = [rng.integers(0, 90, size=nnew).astype(np.int32) for _ in q.rels[rel].cols]
    F2, inserted = oracle.propagate(q, F, rel, new_cols, K, B, SEED32)
    g = grown(q, rel, new_cols)
    # rel's filter equals the filter of its grown rows that pass its children (same size)
    R = g.rels[rel]
    ok = np.ones(R.nrows, dtype=bool)
    if R.pred is not None:
        pc, lo, hi = R.pred
        ok &= (R.cols[pc] >= lo) & (R.cols[pc] < hi)
    for c in t.children[rel]:
        ok &= oracle.bf_probe(F[c][0], R.cols[t.pcol[c]], None, F[c][1], K, B, SEED32)
    rebuilt = oracle.bf_build(R.cols[t.mycol[rel]][ok], None, F[rel][1], K, B, SEED32)
    assert np.array_equal(F2[rel][0], rebuilt)
    # ancestors: a subset of a rebuild's bits; every other filter unchanged
    path = []
    j = rel
    while j != q.root:
        path.append(j)
        j = t.parent[j]
    for j in F:
        if j not in path:
            assert np.array_equal(F2[j][0], F[j][0])
    for j in path[1:]:
        Rj = g.rels[j]
        okj = np.ones(Rj.nrows, dtype=bool)
        if Rj.pred is not None:
            pc, lo, hi = Rj.pred
            okj &= (Rj.cols[pc] >= lo) & (Rj.cols[pc] < hi)
        for c in t.children[j]:
            okj &= oracle.bf_probe(F2[c][0], Rj.cols[t.pcol[c]], None, F2[c][1], K, B, SEED32)
        rb = oracle.bf_build(Rj.cols[t.mycol[j]][okj], None, F[j][1], K, B, SEED32)
        assert np.array_equal(F2[j][0] & ~rb, np.zeros_like(rb))
        assert np.array_equal(F2[j][0] | F[j][0], F2[j][0])
    # no false negatives for the grown query
    tup, cnt, _ = oracle.hash_join(g)
    for j in path:
        if cnt:
            keys = g.rels[j].cols[t.mycol[j]][tup[:, j].astype(np.int64)]
            assert oracle.bf_probe(F2[j][0], keys, None, F2[j][1], K, B, SEED32).all()
    assert inserted[q.root] == 0
