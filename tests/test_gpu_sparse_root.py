"""Materialisation when the root's weighted entries are far apart.

Each block of output finds the root entries covering its outputs and stages their
prefix weights in LDS when they fit (the block's outputs plus two); otherwise its
threads search the root's prefix weights in memory. Here the root's survivors are
mostly false positives of a weak filter (1 bit per key, k = 1): about 1.3M surviving
root rows of which a few hundred have join partners, so every block spans far more
root entries than its LDS window and takes the search in memory, and the odometer steps
over long runs of zero-weight entries. Two relations, and a chain of four with one
weighted path per match. Count, checksum and every tuple against the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from sjtest import check_sorted_in_preorder, lexsort_rows, make_plan

pytestmark = pytest.mark.gpu

WEAK = dict(bits_per_key=1, k=1, block_bits=512, passes=1, seed=51)


def run(q):
    ref, rcnt, rchk = oracle.hash_join(q)
    plan = make_plan(q, **WEAK)
    for _ in range(2):   # recorded, then replayed
        plan.build_filters()
        plan.sieve()
        assert plan.join() == (rcnt, rchk)
        tup = plan.result().cpu().numpy().astype(np.uint32)
        check_sorted_in_preorder(q, tup)
        assert np.array_equal(lexsort_rows(tup), ref)
    return plan, rcnt


def test_two_relations_sparse_root():
    rng = np.random.default_rng(0x5EED0E00)
    n0, n1 = 2_000_000, 60_000
    r1 = rng.integers(0, 2**30, n1).astype(np.int32)
    r0 = rng.integers(2**30, 2**31 - 1, n0).astype(np.int32)   # no partner unless planted
    pos = rng.choice(n0, 500, replace=False)
    r0[pos] = r1[rng.integers(0, n1, 500)]
    q = W.Query("sparse2", [W.Relation("R0", [r0]), W.Relation("R1", [r1])], [(0, 0, 1, 0)], 0)
    plan, cnt = run(q)
    assert plan.survivors(0).shape[0] > 500_000   # mostly zero-weight root entries
    assert 0 < cnt < 2000


def test_chain_of_four_sparse_root():
    rng = np.random.default_rng(0x5EED0E01)
    n0 = 2_000_000
    r0 = [rng.integers(2**30, 2**31 - 1, n0).astype(np.int32)]
    pos = rng.choice(n0, 300, replace=False)
    link = rng.integers(0, 2**30, 300).astype(np.int32)
    r0[0][pos] = link
    # R1 (link -> b), R2 (b -> c), R3 (c): one path per planted link, plus unrelated rows
    def rows(keys_a, n_extra):
        a = np.concatenate([keys_a, rng.integers(0, 2**30, n_extra).astype(np.int32)])
        b = rng.integers(0, 2**30, a.shape[0]).astype(np.int32)
        return a, b
    a1, b1 = rows(link, 20_000)
    a2, b2 = rows(b1[:300], 20_000)
    a3 = np.concatenate([b2[:300], rng.integers(0, 2**30, 20_000).astype(np.int32)])
    q = W.Query("sparse4", [W.Relation("R0", r0), W.Relation("R1", [a1, b1]), W.Relation("R2", [a2, b2]),
                            W.Relation("R3", [a3])], [(0, 0, 1, 0), (1, 1, 2, 0), (2, 1, 3, 0)], 0)
    plan, cnt = run(q)
    assert plan.survivors(0).shape[0] > 500_000
    assert cnt >= 300
