"""DP weights of relations with several children, over many DP tiles, against the oracle.

A relation with c children is weighed with 8 / c entries per thread (8, 4, 2 or 1), and
its DP tile holds 256 threads times that many entries. These cases give the root 2, 3,
4, 5 and 8 children and tens of thousands of surviving root rows, so every DP spans
dozens of tiles with a ragged last one. In the deep case an interior relation has three
children. Dimension keys are permutations (each root row matches at most one row of a
dimension), so the result stays near the number of root survivors while the root's DP
covers every tile. Filters, survivors, count, checksum and every tuple must equal the
oracle's, through recorded graphs and eagerly.
"""
import numpy as np
import pytest

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import check_sieve, check_sorted_in_preorder, lexsort_rows, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=31)


def run(q):
    ref, rcnt, rchk = oracle.hash_join(q)
    rels = to_device(q)
    for eager in (False, True):
        plan = sj.Plan(sj.Context(0), rels, q.edges, root=q.root, eager=eager, **OPTS)
        for _ in range(1 if eager else 2):
            plan.build_filters()
            plan.sieve()
            S, _ = check_sieve(q, plan, **OPTS)
            assert plan.join() == (rcnt, rchk)
            tup = plan.result().cpu().numpy().astype(np.uint32)
            check_sorted_in_preorder(q, tup)
            assert np.array_equal(lexsort_rows(tup), ref)
    return rcnt, S


@pytest.mark.parametrize("ndims,fact_rows", [(2, 70001), (3, 60013), (4, 50021), (5, 45007), (8, 40009)])
def test_root_with_many_children(ndims, fact_rows):
    q = W.star(fact_rows, ndims, 20011, 0.93, 0x5EED0D00 + ndims)
    cnt, S = run(q)
    # enough root survivors for dozens of DP tiles at this fan-out (tile = 256 * 8 / ndims')
    per_thread = 8 if ndims <= 1 else 4 if ndims == 2 else 2 if ndims <= 4 else 1
    assert S[0].shape[0] > 20 * 256 * per_thread
    assert cnt > 0


def test_interior_relation_with_three_children():
    """0 - 1, 1 - {2, 3, 4}, 0 - 5: relation 1 is weighed with 2 entries per thread
    over its buckets, the root with 4."""
    rng = np.random.default_rng(0x5EED0D10)
    n0, n1, nd = 60000, 40000, 30011
    r0 = [rng.integers(0, n1, n0).astype(np.int32), rng.integers(0, nd, n0).astype(np.int32)]
    r1 = [rng.permutation(n1).astype(np.int32)] + [rng.integers(0, nd, n1).astype(np.int32) for _ in range(3)]
    dims = [[rng.permutation(nd).astype(np.int32)] for _ in range(4)]
    rels = [W.Relation("R0", r0), W.Relation("R1", r1, pred=(1, 0, int(nd * 0.95)))]
    rels += [W.Relation("D%d" % i, d) for i, d in enumerate(dims)]
    edges = [(0, 0, 1, 0), (1, 1, 2, 0), (1, 2, 3, 0), (1, 3, 4, 0), (0, 1, 5, 0)]
    q = W.Query("fan3", rels, edges, 0)
    cnt, S = run(q)
    assert S[1].shape[0] > 20 * 512
    assert cnt > 20 * 512


def test_tile_scan_over_several_rounds():
    """Five children (one entry per thread, 256-entry tiles) and about 600K root
    survivors: more than 2048 DP tiles, so the tile-sum scan takes several rounds."""
    q = W.star(700_001, 5, 20011, 0.97, 0x5EED0D20)
    cnt, S = run(q)
    assert S[0].shape[0] > 2048 * 256
