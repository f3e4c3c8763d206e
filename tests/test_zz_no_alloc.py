"""sj_bind_static_workspace: plans bound to the library's static workspace (no device
allocation by the caller or the library) give exactly what the same plans give on a
caller workspace (sj_bind_workspace), through the C ABI: survivors, every filter word,
count, checksum and tuples, on two calls in a row on the same static workspace, the
second with a smaller input. A plan larger than the static workspace is refused."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import check_sieve, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=10, k=7, block_bits=512, passes=2, seed=0x5EED0001)


def outputs(plan, q):
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    tup = plan.result().cpu().numpy().copy()
    surv = [plan.survivors(i).cpu().numpy().copy() for i in range(len(q.rels))]
    words = [plan.filter_words(f).cpu().numpy().copy() for f in range(plan.filter_count())]
    return cnt, chk, tup, surv, words


def compare(q):
    rels = to_device(q)
    ctx = sj.Context(0)
    ref = outputs(sj.Plan(ctx, rels, q.edges, **OPTS), q)          # caller workspace
    st = sj.Plan(ctx, rels, q.edges, static_workspace=True, **OPTS)
    assert st.workspace is None and st.workspace_bytes <= sj.SJ_STATIC_WORKSPACE_BYTES
    got = outputs(st, q)
    assert got[:2] == ref[:2]
    assert np.array_equal(got[2], ref[2])
    for a, b in zip(got[3], ref[3]):
        assert np.array_equal(a, b)
    for a, b in zip(got[4], ref[4]):
        assert np.array_equal(a, b)
    check_sieve(q, st, **OPTS)
    _, rcnt, rchk = oracle.hash_join(q)
    assert got[:2] == (rcnt, rchk)
    return got[0]


def test_static_workspace_equals_caller_workspace_twice_smaller_second():
    big = W.config1(scale=2.0)     # 3 x 200,000 rows: a workspace of 52 of the 64 MiB
    small = W.config1(seed=0x5EED0011, scale=0.1)
    assert compare(big) > 0
    assert compare(small) > 0


def test_plan_larger_than_the_static_workspace_is_refused():
    q = W.config1(scale=4.0)       # 3 x 400,000 rows
    ctx = sj.Context(0)
    with pytest.raises(sj.SjError) as e:
        sj.Plan(ctx, to_device(q), q.edges, static_workspace=True, **OPTS)
    assert e.value.code == sj.SJ_ERR_NOMEM
    assert "static workspace" in ctx.last_error()
