"""The factorised materialisation against the oracle.

Every non-root relation with children gets a table of the tuples below each of its
entries (in its sort scratch), deepest first; the output is one expansion of the
root. These cases check the tuples (sorted in preorder and equal to the oracle's),
synchronously and asynchronously, in row ids and projected values:
- chains whose middle tables fit, and one whose table does not (a relation of ten rows
  fanning out to two hundred), where the per-tuple decode writes the output instead;
- trees with two and four children below a non-root relation (mixed-radix digits in
  the tables), a bushy tree with tables at two depths, a star of four leaves (no
  tables), a star of six (more children than the tables take: the decode alone);
- a single relation, and an empty result.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import check_sorted_in_preorder, lexsort_rows, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=5)


def tree(parents, rows, domain, seed, pcols=None):
    """Relation i > 0 joins parents[i] on column pcols[i] (default i % 2) of the parent
    and column 0 of itself; two int32 columns each."""
    rng = np.random.default_rng(seed)
    rels = [W.Relation("R%d" % i, [rng.integers(0, domain, n).astype(np.int32) for _ in range(2)])
            for i, n in enumerate(rows)]
    pc = pcols or [i % 2 for i in range(len(rows))]
    edges = [(parents[i], pc[i], i, 0) for i in range(1, len(rows))]
    return W.Query("tree", rels, edges, 0)


def check(q, values=True):
    ref, rc, rk = oracle.hash_join(q)
    rels = to_device(q)
    p = sj.Plan(sj.Context(0), rels, q.edges, root=q.root, **OPTS)
    for _ in range(2):   # recorded, then replayed
        p.build_filters()
        p.sieve()
        assert p.join() == (rc, rk)
        tup = p.result().cpu().numpy().astype(np.uint32)
        check_sorted_in_preorder(q, tup)
        assert np.array_equal(lexsort_rows(tup), ref)
        if values:
            got = p.result(mode=sj.SJ_VALUES).cpu().numpy()
            assert np.array_equal(got, oracle.project(q, tup))
    # asynchronous count and result (the count stays on the device)
    p.build_filters()
    p.sieve()
    p.join_async()
    out = torch.full((rc + 3, len(q.rels)), -7, dtype=torch.int32, device="cuda:0")
    p.result_async(out)
    assert p.join_wait()[:2] == (rc, rk)
    got = out.cpu().numpy()
    assert (got[rc:] == -7).all()
    assert np.array_equal(got[:rc].astype(np.uint32), tup)
    return rc


@pytest.mark.parametrize("seed", range(6))
def test_chains(seed):
    n = 3 + seed % 4
    q = tree(list(range(-1, n - 1)), [int(x) for x in np.random.default_rng(seed).integers(200, 3000, n)], 150,
             0x3A7 + seed)
    check(q)


def test_table_too_large_for_its_scratch():
    """R1 has ten rows, all on one key, and R2 two hundred rows on the key they lead to:
    R1's table would hold 2000 rows of two words in scratch sized for ten rows."""
    r0 = W.Relation("R0", [np.arange(5, dtype=np.int32), np.full(5, 7, np.int32)])
    r1 = W.Relation("R1", [np.full(10, 7, np.int32), np.full(10, 9, np.int32)])
    r2 = W.Relation("R2", [np.full(200, 9, np.int32), np.arange(200, dtype=np.int32)])
    q = W.Query("fanout", [r0, r1, r2], [(0, 1, 1, 0), (1, 1, 2, 0)], 0)
    assert check(q) == 5 * 10 * 200
    # the same shape with a table that fits (one row below each R1 entry)
    r2s = W.Relation("R2", [np.full(1, 9, np.int32), np.arange(1, dtype=np.int32)])
    assert check(W.Query("fits", [r0, r1, r2s], [(0, 1, 1, 0), (1, 1, 2, 0)], 0)) == 50


def test_two_and_four_children_below_a_non_root_relation():
    #    0
    #    1
    #  2   3          (two children of 1: its table's rows are mixed-radix)
    q = tree([-1, 0, 1, 1], [600, 500, 400, 300], 60, 0x3B1, pcols=[0, 1, 1, 0])
    check(q)
    #      0
    #      1
    #  2  3  4  5     (four)
    q = tree([-1, 0, 1, 1, 1, 1], [300, 200, 60, 50, 40, 30], 12, 0x3B2, pcols=[0, 1, 0, 1, 0, 1])
    check(q)


def test_bushy_tables_at_two_depths():
    #        0
    #     1     2
    #    3 4     5
    #    6       7
    q = tree([-1, 0, 0, 1, 1, 2, 3, 5], [700, 400, 500, 300, 200, 300, 250, 200], 90, 0x3B3)
    check(q)


def test_stars():
    check(W.star(20000, 4, 1000, 0.5, 0x3B4))
    check(W.star(8000, 6, 300, 0.7, 0x3B5))   # six children of the root: the decode alone


def test_single_relation_and_empty():
    r = W.Relation("R0", [np.arange(100, dtype=np.int32), np.arange(100, dtype=np.int32)])
    q = W.Query("one", [r], [], 0)
    ref, rc, rk = oracle.hash_join(q)
    p = sj.Plan(sj.Context(0), to_device(q), q.edges, **OPTS)
    p.build_filters()
    p.sieve()
    assert p.join() == (rc, rk) == (100, rk)
    assert np.array_equal(p.result().cpu().numpy().astype(np.uint32), ref)
    a = W.Relation("A", [np.zeros(50, np.int32), np.ones(50, np.int32)])
    b = W.Relation("B", [np.full(40, 2, np.int32), np.ones(40, np.int32)])
    c = W.Relation("C", [np.ones(30, np.int32), np.ones(30, np.int32)])
    assert check(W.Query("empty", [a, b, c], [(0, 1, 1, 0), (1, 1, 2, 0)], 0)) == 0
