"""3-cycles counted by intersection (the default count pass of a 3-cycle query).

Every case is checked three ways: the intersection count, the binary plan's count
(SJ_FLAG_BINARY_CYCLES) and the oracle's binary hash join agree on count and
checksum, and the tuples written by the intersection walk and by the binary plan
(each compared as a sorted multiset; the binary plan's also sorted in preorder) equal
the oracle's. Cases: random small 3-cycles
(empty relations, several columns, negative and extreme keys, repeated pairs), the
pair whose 64-bit key equals the hash's empty marker, predicates, three different
edge relations, the power-law triangle at reduced size, the asynchronous count,
graph replays, and the full-size triangle workload (50M edges) with a sampled first
relation, checked against the oracle's adjacency-intersection count over that sample.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import check_sorted_in_preorder, lexsort_rows, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=7)


def counts(q, rels=None, **kw):
    rels = rels if rels is not None else to_device(q)
    p = sj.Plan(sj.Context(0), rels, q.edges, root=q.root, **dict(OPTS, **kw))
    p.build_filters()
    p.sieve()
    return p, p.join()


def used_intersection(q, rels):
    p = sj.Plan(sj.Context(0), rels, q.edges, root=q.root, profile=True, **OPTS)
    p.build_filters()
    p.sieve()
    p.join()
    return any(e["label"] == "tri_count" for e in p.profile())


def check_all(q, expect_tri=True):
    rels = to_device(q)
    ref, rcnt, rchk = oracle.hash_join(q)
    p, cc = counts(q, rels)
    _, cb = counts(q, rels, binary_cycles=True)
    assert cc == (rcnt, rchk), (q.name, cc, (rcnt, rchk))
    assert cb == (rcnt, rchk)
    assert used_intersection(q, rels) == expect_tri
    # the intersection walk writes the tuples (in walk order); the binary plan decodes its
    # own count pass (sorted in preorder)
    tup = p.result().cpu().numpy().astype(np.uint32)
    assert np.array_equal(lexsort_rows(tup), lexsort_rows(ref))
    pb, _ = counts(q, rels, binary_cycles=True)
    tb = pb.result().cpu().numpy().astype(np.uint32)
    assert np.array_equal(lexsort_rows(tb), lexsort_rows(ref))
    check_sorted_in_preorder(q, tb)
    return rcnt


def three_cycles():
    out = []
    for seed in range(40):
        for kind in ("triangle", "selfjoin"):
            q = W.tiny_random(seed, kind=kind)
            if len(q.edges) == 3:
                out.append(pytest.param(q, id="%s-%d" % (kind, seed)))
    return out


@pytest.mark.parametrize("q", three_cycles())
def test_small_random_three_cycles(q):
    check_all(q)


def test_the_empty_marker_pair():
    """Every key is -1, so every (key, key) pair is 0xFFFF_FFFF_FFFF_FFFF: all n1 n2 n3
    tuples match through the hash's spare slot."""
    m1 = np.full(7, -1, np.int32)
    rels = [W.Relation("A", [m1.copy(), m1.copy()]), W.Relation("B", [np.full(5, -1, np.int32)] * 2),
            W.Relation("C", [np.full(3, -1, np.int32), np.full(3, -1, np.int32)])]
    q = W.Query("allneg", rels, [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 0, 0)], 0)
    assert check_all(q) == 7 * 5 * 3


def test_repeated_pairs_and_mixed_keys():
    """Many copies of the same (key, key) pair in each relation, extreme keys."""
    rng = np.random.default_rng(5)
    vals = np.array([-2**31, 2**31 - 1, -1, 0, 1, 2], np.int32)
    rels = [W.Relation(n, [vals[rng.integers(0, 6, 400)], vals[rng.integers(0, 6, 400)]]) for n in "ABC"]
    q = W.Query("rep", rels, [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 0, 0)], 0)
    assert check_all(q) > 0


def test_power_law_triangle_with_predicates_and_distinct_tables():
    q = W.triangle(30000, 2000, 2.1, 0x5EED00E1)
    check_all(q)
    # a predicate on each instance (on the edge's own columns)
    qp = W.Query("pred", [W.Relation(r.name, r.cols, (i % 2, 0, 1400)) for i, r in enumerate(q.rels)], q.edges, 0)
    check_all(qp)
    # three different edge relations, other column order on the middle one
    a = W.triangle(20000, 1500, 2.1, 11).rels[0]
    b = W.triangle(20000, 1500, 2.1, 12).rels[0]
    c = W.triangle(20000, 1500, 2.1, 13).rels[0]
    q3 = W.Query("three", [W.Relation("A", a.cols), W.Relation("B", [b.cols[1], b.cols[0]]),
                           W.Relation("C", c.cols)], [(0, 1, 1, 1), (1, 0, 2, 0), (2, 1, 0, 0)], 0)
    check_all(q3)


def test_four_cycles_keep_the_binary_plan():
    q = W.tiny_random(31, kind="cycle4")
    rels = to_device(q)
    assert not used_intersection(q, rels)


def test_async_count_and_graph_replays():
    q = W.triangle(40000, 2500, 2.1, 0x5EED00E2)
    rels = to_device(q)
    rc, rk = oracle.triangle_cycles(*q.rels[0].cols)
    p = sj.Plan(sj.Context(0), rels, q.edges, **OPTS)
    for _ in range(3):   # recorded on the first call, replayed after
        p.build_filters()
        p.sieve()
        p.join_async()
        assert p.join_wait()[:2] == (rc, rk)
        p.build_filters()
        p.sieve()
        assert p.join() == (rc, rk)
    with pytest.raises(sj.SjError) as e:
        p.result_async(torch.empty((rc + 1, 3), dtype=torch.int32, device="cuda:0"))
    assert e.value.code == sj.SJ_ERR_UNSUPPORTED


@pytest.fixture(scope="module")
def full_edges():
    t = time.time()
    q = W.config4(scale=1.0, device="cuda:0")
    print("\n# full-size triangle workload: %d edges generated in %.1f s" % (q.rels[0].nrows, time.time() - t),
          flush=True)
    return q


def test_full_size_triangle_sampled_first_relation(full_edges):
    """E1 = 600 sampled edges, E2 = E3 = the whole 50M-edge relation: the plan's
    capacities, hashes and launch grids are the full-size ones and the oracle's
    adjacency-intersection count over the sample is affordable."""
    src, dst = full_edges.rels[0].cols
    idx = np.sort(np.random.default_rng(0x5EED00E3).choice(src.shape[0], 600, replace=False))
    rels = [W.Relation("S", [src[idx], dst[idx]]), W.Relation("E2", [src, dst]), W.Relation("E3", [src, dst])]
    q = W.Query("sample", rels, [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 0, 0)], 0)
    dev = to_device(q)
    t = time.time()
    _, cc = counts(q, dev)
    print("# GPU plan over the sample: %.1f s" % (time.time() - t), flush=True)
    t = time.time()
    rc, rk = oracle.triangle_cycles(src, dst, e1=(src[idx], dst[idx]))
    print("# oracle: %.1f s, %d tuples" % (time.time() - t, rc), flush=True)
    assert cc == (rc, rk)
    assert rc > 0
