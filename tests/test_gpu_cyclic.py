"""Cyclic joins of any shape through the binary plan.

The plan enumerates the spanning tree without its last preorder relation L and matches
L per prefix: L is sorted by the column of the first closing edge that ends at it,
other closing edges at L are checked on each entry of the matching run, and closing
edges between two other relations are checked on the prefix. Every case compares
count, checksum, every tuple (row ids and projected values) with the oracle's binary
hash join, which checks every closing edge on the enumerated tuples: random connected
graphs with one to four extra edges over three to six relations (several columns per
relation, so that closing edges land on different columns, repeated keys, predicates,
empty relations), a 4-cycle with a chord, two triangles sharing a relation, closing
edges on two columns of L, and one and two passes, in recorded-graph and eager plans.
"""
import numpy as np
import pytest

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import check_sieve, check_sorted_in_preorder, lexsort_rows, to_device

pytestmark = pytest.mark.gpu


def random_cyclic(seed):
    rng = np.random.default_rng(0xC7C + seed)
    n = int(rng.integers(3, 7))
    ncols = 3
    rels = []
    for i in range(n):
        rows = 0 if (seed % 17 == 5 and i == n - 1) else int(rng.integers(4, 60))
        dom = int(rng.integers(2, 7))
        cols = [rng.integers(-2, dom, rows).astype(np.int32) for _ in range(ncols)]
        pred = (2, -1, dom - 1) if rng.random() < 0.3 else None
        rels.append(W.Relation("R%d" % i, cols, pred))
    edges = []
    for i in range(1, n):   # a random spanning tree
        j = int(rng.integers(0, i))
        edges.append((j, int(rng.integers(0, ncols)), i, int(rng.integers(0, ncols))))
    extra = int(rng.integers(1, 5))
    have = {(a, b) for a, _, b, _ in edges}
    for _ in range(extra):
        a, b = sorted(int(x) for x in rng.choice(n, size=2, replace=False))
        edges.append((a, int(rng.integers(0, ncols)), b, int(rng.integers(0, ncols))))
    return W.Query("cyc%d" % seed, rels, edges, 0)


def check(q, passes=2, eager=False, sorted_result=True):
    ref, rcnt, rchk = oracle.hash_join(q)
    plan = sj.Plan(sj.Context(0), to_device(q), q.edges, root=q.root, eager=eager, bits_per_key=4, k=3,
                   passes=passes, seed=3, binary_cycles=True)
    for _ in range(2):
        plan.build_filters()
        plan.sieve()
        check_sieve(q, plan, 4, 3, 512, passes, 3)
        assert plan.join() == (rcnt, rchk)
        tup = plan.result().cpu().numpy().astype(np.uint32)
        assert np.array_equal(lexsort_rows(tup), ref)
        if sorted_result:
            check_sorted_in_preorder(q, tup)
        vals = plan.result(mode=sj.SJ_VALUES).cpu().numpy()
        assert np.array_equal(vals, oracle.project(q, tup))
    return rcnt


@pytest.mark.parametrize("seed", range(48))
def test_random_cyclic_shapes(seed):
    q = random_cyclic(seed)
    check(q, passes=1 + seed % 2, eager=seed % 3 == 0)


def chain_rels(n, rows, dom, seed, ncols=3):
    rng = np.random.default_rng(seed)
    return [W.Relation("R%d" % i, [rng.integers(0, dom, rows).astype(np.int32) for _ in range(ncols)])
            for i in range(n)]


def test_four_cycle_with_a_chord():
    rels = chain_rels(4, 300, 12, 1)
    edges = [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 3, 0), (3, 1, 0, 0), (0, 2, 2, 2)]
    assert check(W.Query("chord", rels, edges, 0)) > 0


def test_two_triangles_sharing_a_relation():
    rels = chain_rels(5, 250, 10, 2)
    edges = [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 0, 0),     # triangle 0-1-2
             (0, 2, 3, 0), (3, 1, 4, 0), (4, 1, 0, 2)]     # triangle 0-3-4 on another column of 0
    assert check(W.Query("bowtie", rels, edges, 0)) > 0


def test_closing_edges_on_two_columns_of_the_last_relation():
    rels = chain_rels(3, 400, 8, 3)
    edges = [(0, 1, 1, 0), (1, 1, 2, 0), (0, 0, 2, 1), (1, 2, 2, 2)]
    assert check(W.Query("twocols", rels, edges, 0)) > 0


def test_closing_edge_on_the_tree_column_of_the_last_relation():
    rels = chain_rels(3, 300, 6, 4)
    edges = [(0, 1, 1, 0), (1, 1, 2, 0), (0, 2, 2, 0)]   # the closing edge reads L's tree column
    assert check(W.Query("samecol", rels, edges, 0)) > 0
