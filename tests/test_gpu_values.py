"""Value tuples (SJ_VALUES): the join result written as column values instead of row
ids, checked element by element against oracle.project of the oracle's result.

GPU tuples of chains and stars come in relation-index order, as the oracle's sorted
tuples do, so values are compared row for row with oracle.project(oracle result). For
shapes whose enumeration order is another preorder (trees, cycles) the row-id result is
first checked against the oracle as a sorted multiset, then the value result against
oracle.project of the GPU's own row ids (the same order). Both the synchronous and the
asynchronous materialisation are covered, with the default projection (every column of
every relation) and chosen ones.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import lexsort_rows, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=11)


def run(q, proj=None, eager=False, **opts):
    plan = sj.Plan(sj.Context(0), to_device(q), q.edges, root=q.root, eager=eager, **dict(OPTS, **opts))
    if proj is not None:
        plan.set_projection(proj)
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    rids = plan.result().cpu().numpy().astype(np.uint32)
    vals = plan.result(mode=sj.SJ_VALUES).cpu().numpy()
    return plan, cnt, chk, rids, vals


@pytest.mark.parametrize("proj", [None, [(2, 1), (0, 0), (1, 1), (1, 0)], [(1, 1)]])
def test_chain_values(proj):
    q = W.chain(3, [9000, 7000, 8000], 3000, 0.6, 0x5EED0A01)
    ref, rcnt, rchk = oracle.hash_join(q)
    plan, cnt, chk, rids, vals = run(q, proj)
    assert (cnt, chk) == (rcnt, rchk)
    assert np.array_equal(rids, ref)
    want = oracle.project(q, ref, proj)
    assert vals.shape == want.shape and np.array_equal(vals, want)
    assert plan.footprint(sj.SJ_VALUES)["result_bytes"] == want.size * 4


def test_star_values_with_predicates_async():
    q = W.star(200_000, 4, 5000, 0.3, 0x5EED0A02)
    ref, rcnt, rchk = oracle.hash_join(q)
    plan = sj.Plan(sj.Context(0), to_device(q), q.edges, root=q.root, **OPTS)
    want = oracle.project(q, ref)
    out = torch.full((rcnt + 5, plan.width(sj.SJ_VALUES)), -7, dtype=torch.int32, device="cuda:0")
    for _ in range(3):   # recorded graphs, replayed
        plan.build_filters()
        plan.sieve()
        plan.join_async()
        plan.result_async(out, mode=sj.SJ_VALUES)
        assert plan.join_wait() == (rcnt, rchk, sj.SJ_OK)
        got = out.cpu().numpy()
        assert np.array_equal(got[:rcnt], want)
        assert (got[rcnt:] == -7).all()
    # a buffer one tuple short: nothing written, status says so
    small = torch.full((rcnt - 1, plan.width(sj.SJ_VALUES)), -3, dtype=torch.int32, device="cuda:0")
    plan.build_filters()
    plan.sieve()
    plan.join_async()
    plan.result_async(small, mode=sj.SJ_VALUES)
    assert plan.join_wait() == (rcnt, rchk, sj.SJ_ERR_CAPACITY)
    assert (small.cpu().numpy() == -3).all()


@pytest.mark.parametrize("seed", range(12))
def test_random_shapes_values(seed):
    q = W.tiny_random(0x5EED0A10 + seed)
    ref, rcnt, rchk = oracle.hash_join(q)
    try:
        plan, cnt, chk, rids, vals = run(q)
    except sj.SjError as e:
        assert e.code == sj.SJ_ERR_UNSUPPORTED   # a cyclic shape this build does not execute
        return
    assert (cnt, chk) == (rcnt, rchk)
    assert np.array_equal(lexsort_rows(rids), ref)
    assert np.array_equal(vals, oracle.project(q, rids))


@pytest.mark.parametrize("binary", [False, True])
def test_cycle_values(binary):
    q = W.chain(4, 3000, 400, 0.3, 0x5EED0A03)
    q.edges.append((3, 1, 0, 0))   # close the chain into a 4-cycle
    ref, rcnt, rchk = oracle.hash_join(q)
    plan, cnt, chk, rids, vals = run(q, proj=[(3, 1), (0, 0), (2, 0)], binary_cycles=binary)
    assert (cnt, chk) == (rcnt, rchk) and rcnt > 0
    assert np.array_equal(lexsort_rows(rids), ref)
    assert np.array_equal(vals, oracle.project(q, rids, [(3, 1), (0, 0), (2, 0)]))


def test_triangle_values():
    q = W.triangle(20000, 2000, 2.1, 0x5EED0A04)
    ref, rcnt, rchk = oracle.hash_join(q)
    plan, cnt, chk, rids, vals = run(q)
    assert (cnt, chk) == (rcnt, rchk) and rcnt > 0
    assert np.array_equal(lexsort_rows(rids), ref)
    assert np.array_equal(vals, oracle.project(q, rids))


def test_projection_too_wide_is_refused():
    rels = [W.Relation("R%d" % i, [np.arange(50, dtype=np.int32) % 7 for _ in range(17)]) for i in range(2)]
    q = W.Query("wide", rels, [(0, 0, 1, 0)], 0)
    plan = sj.Plan(sj.Context(0), to_device(q), q.edges, **OPTS)
    plan.build_filters()
    plan.sieve()
    plan.join()
    with pytest.raises(sj.SjError) as e:
        plan.result(mode=sj.SJ_VALUES)
    assert e.value.code == sj.SJ_ERR_UNSUPPORTED
    plan.set_projection([(1, 16), (0, 3)])
    ref, _, _ = oracle.hash_join(q)
    assert np.array_equal(plan.result(mode=sj.SJ_VALUES).cpu().numpy(), oracle.project(q, ref, [(1, 16), (0, 3)]))
