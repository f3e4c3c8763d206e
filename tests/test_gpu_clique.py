"""4-cliques counted by intersection (the count pass of every 4-clique query).

Every case checks the GPU count and checksum against the oracle's generic join over
the four variables (oracle.clique4, pinned by brute force, closed forms and the
binary plan), and at small sizes also against the oracle's binary hash join. The
sieve in front of the walk is checked against oracle.sieve (survivors and filters
bit for bit). Cases: tiny random relations (empty relations, repeated pairs, self
loops, negative and extreme keys, an unused extra column), the pair equal to the pair
hash's empty marker, complete and transitive digraphs (closed forms), predicates,
relabelled queries (relation order, column order, root), one pass, the asynchronous
count and graph replays, and the vote-network-sized workload against the oracle's
stored value, with the 3-clique on the same graph (the 3-cycle path). The tuples
come from the walk too (in walk order): at small sizes they equal the oracle's as
a sorted multiset, in row ids and projected values; at the vote-network size every
tuple satisfies every edge and their checksum is the oracle's. The binary plan
(SJ_FLAG_BINARY_CYCLES) reaches the same count, checksum and tuples; the asynchronous
result refuses cyclic joins.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import check_sieve, lexsort_rows, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=7)


def run(q, rels=None, **kw):
    rels = rels if rels is not None else to_device(q)
    p = sj.Plan(sj.Context(0), rels, q.edges, root=q.root, **dict(OPTS, **kw))
    p.build_filters()
    p.sieve()
    return p, p.join()


def used_k4(q, rels):
    p = sj.Plan(sj.Context(0), rels, q.edges, root=q.root, profile=True, **OPTS)
    p.build_filters()
    p.sieve()
    p.join()
    return any(e["label"] == "k4_count" for e in p.profile())


def check(q, binary_too=True):
    rels = to_device(q)
    want = oracle.clique4(q)
    p, got = run(q, rels)
    assert got == want, (q.name, got, want)
    tup = p.result().cpu().numpy().astype(np.uint32)
    if binary_too:
        ref, bc, bk = oracle.hash_join(q)
        assert (bc, bk) == want
        assert np.array_equal(lexsort_rows(tup), lexsort_rows(ref))
        assert np.array_equal(lexsort_rows(p.result(mode=sj.SJ_VALUES).cpu().numpy()),
                              lexsort_rows(oracle.project(q, tup)))
    else:
        check_tuples(q, tup, *want)
    return want[0]


def check_tuples(q, tup, count, checksum):
    """Every tuple satisfies every join edge; count and checksum are the oracle's."""
    assert tup.shape[0] == count
    t = tup.astype(np.int64)
    for a, ca, b, cb in q.edges:
        assert np.array_equal(np.asarray(q.rels[a].cols[ca])[t[:, a]], np.asarray(q.rels[b].cols[cb])[t[:, b]])
    assert oracle.checksum_of(tup) == checksum


def tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    vals = np.array([-2**31, 2**31 - 1, -1, 0, 1, 2, 3], np.int32)
    rels = []
    for i, name in enumerate(("AB", "AC", "AD", "BC", "BD", "CD")):
        n = int(rng.integers(0, 14)) if seed % 5 else int(rng.integers(1, 14))
        pick = rng.integers(3, 7) if seed % 3 else 7
        cols = [vals[rng.integers(0, pick, n)] for _ in range(2)]
        if seed % 4 == 1:
            cols.append(rng.integers(-5, 5, n).astype(np.int32))   # a column no edge uses
        rels.append(W.Relation(name, cols))
    return W.Query("tiny%d" % seed, rels, list(W.CLIQUE4_EDGES), 0)


@pytest.mark.parametrize("seed", range(40))
def test_tiny_random_cliques(seed):
    check(tiny(seed))


def test_the_empty_marker_pair():
    """Every key is -1: every pair is 0xFFFF_FFFF_FFFF_FFFF, the hash's empty marker,
    held in its spare slot; every combination of rows matches."""
    sizes = [2, 3, 2, 1, 2, 3]
    rels = [W.Relation(n, [np.full(m, -1, np.int32), np.full(m, -1, np.int32)])
            for n, m in zip(("AB", "AC", "AD", "BC", "BD", "CD"), sizes)]
    q = W.Query("allneg", rels, list(W.CLIQUE4_EDGES), 0)
    assert check(q) == int(np.prod(sizes))


def complete(n, transitive):
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v and (u < v or not transitive)]
    return (np.array([p[0] for p in pairs], np.int32), np.array([p[1] for p in pairs], np.int32))


@pytest.mark.parametrize("n", [4, 9, 17])
def test_closed_forms(n):
    assert check(W.clique4(*complete(n, False)), binary_too=n < 10) == n * (n - 1) * (n - 2) * (n - 3)
    assert check(W.clique4(*complete(n, True)), binary_too=n < 10) == n * (n - 1) * (n - 2) * (n - 3) // 24


def test_power_law_with_predicates_relabelling_and_one_pass():
    s, d = W.powerlaw_edges(3000, 300, 2.3, 0xC4A)
    q = W.clique4(s, d)
    assert check(q) > 0
    assert used_k4(q, to_device(q))
    qp = W.Query("pred", [W.Relation(r.name, r.cols, (i % 2, 0, 220)) for i, r in enumerate(q.rels)], q.edges, 0)
    check(qp)
    # another relation order, swapped columns, another root
    perm = [3, 5, 0, 2, 4, 1]
    inv = {old: new for new, old in enumerate(perm)}
    rels = [None] * 6
    for old, new in inv.items():
        rels[new] = W.Relation(q.rels[old].name, [q.rels[old].cols[1], q.rels[old].cols[0]])
    edges = [(inv[a], 1 - ca, inv[b], 1 - cb) for a, ca, b, cb in q.edges]
    for root in (0, 4):
        check(W.Query("relabelled", rels, edges, root))
    rels1 = to_device(q)
    _, got = run(q, rels1, passes=1)
    assert got == oracle.clique4(q)


@pytest.mark.parametrize("passes", [1, 2])
def test_sieve_in_front_of_the_walk(passes):
    s, d = W.powerlaw_edges(4000, 400, 2.3, 0xC4B)
    q = W.clique4(s, d)
    p, _ = run(q, passes=passes)
    check_sieve(q, p, OPTS["bits_per_key"], OPTS["k"], OPTS["block_bits"], passes, OPTS["seed"])


def test_async_count_graph_replays_and_refusals():
    s, d = W.powerlaw_edges(5000, 500, 2.3, 0xC4C)
    q = W.clique4(s, d)
    want = oracle.clique4(q)
    rels = to_device(q)
    p = sj.Plan(sj.Context(0), rels, q.edges, **OPTS)
    for _ in range(3):   # recorded on the first call, replayed after
        p.build_filters()
        p.sieve()
        p.join_async()
        assert p.join_wait()[:2] == want
        p.build_filters()
        p.sieve()
        assert p.join() == want
    ref, _, _ = oracle.hash_join(q)
    for _ in range(2):
        out = torch.full((want[0] + 1, 6), -7, dtype=torch.int32, device="cuda:0")
        p.result(out)
        got = out.cpu().numpy()
        assert (got[-1] == -7).all()
        assert np.array_equal(lexsort_rows(got[:-1].astype(np.uint32)), lexsort_rows(ref))
    with pytest.raises(sj.SjError) as e:
        p.result(torch.empty((want[0] - 1, 6), dtype=torch.int32, device="cuda:0"))
    assert e.value.code == sj.SJ_ERR_CAPACITY
    with pytest.raises(sj.SjError) as e:
        p.result_async(torch.empty((want[0] + 1, 6), dtype=torch.int32, device="cuda:0"))
    assert e.value.code == sj.SJ_ERR_UNSUPPORTED
    # the binary plan (spanning tree, closing edges checked per prefix and per entry of
    # the last relation) reaches the same result, tuples sorted in preorder
    b = sj.Plan(sj.Context(0), rels, q.edges, binary_cycles=True, **OPTS)
    b.build_filters()
    b.sieve()
    assert b.join() == want
    tb = b.result().cpu().numpy().astype(np.uint32)
    assert np.array_equal(lexsort_rows(tb), lexsort_rows(ref))


def test_vote_network_sized_cliques():
    with open(os.path.join(os.path.dirname(__file__), "golden", "clique_wiki.json")) as fh:
        doc = json.load(fh)
    q4 = W.config6(k=4)
    assert q4.rels[0].nrows == doc["edges"]
    rels = to_device(q4)
    p, got = run(q4, rels)
    assert got == (doc["clique4"]["count"], doc["clique4"]["checksum"])
    check_tuples(q4, p.result().cpu().numpy().astype(np.uint32), *got)
    q3 = W.config6(k=3)
    p3, got3 = run(q3, to_device(q3))
    assert got3 == (doc["clique3"]["count"], doc["clique3"]["checksum"])
    check_tuples(q3, p3.result().cpu().numpy().astype(np.uint32), *got3)
