"""Results past 32 bits: counts, checksums and output positions beyond 2^32 tuples.

- Two relations on one key, 65,537 x 65,539 rows: 4,295,229,443 result tuples (34 GB of
  output). The count is the product, the checksum the oracle's sum-product DP, and every
  tuple is checked on the device against its closed form: the tuples come in the order
  of the root's rows, each with all of the other relation's rows in row order, so tuple
  t is (t // n1, t % n1). A buffer one tuple short is refused and nothing is written.
- A chain of three relations whose result has about 10^12 tuples, counted only
  (synchronously and asynchronously), against the product and the oracle's DP.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import make_plan

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=41)


def test_tuples_past_two_to_the_32():
    n0, n1 = 65537, 65539
    q = W.Query("pair", [W.Relation("R0", [np.full(n0, 5, np.int32)]),
                         W.Relation("R1", [np.full(n1, 5, np.int32)])], [(0, 0, 1, 0)], 0)
    plan = make_plan(q, **OPTS)
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    assert cnt == n0 * n1 and cnt > 2**32
    assert (cnt, chk) == oracle.join_tree_dp(q)
    dev = torch.device("cuda:0")
    out = torch.full((cnt, 2), -1, dtype=torch.int32, device=dev)
    with pytest.raises(sj.SjError) as e:
        plan.result(out[:cnt - 1])
    assert e.value.code == sj.SJ_ERR_CAPACITY
    assert int(out[0, 0]) == -1 and int(out[-1, 1]) == -1   # nothing written
    plan.result(out)
    torch.cuda.synchronize()
    chunk = 1 << 28
    for t0 in range(0, cnt, chunk):
        t1 = min(cnt, t0 + chunk)
        t = torch.arange(t0, t1, dtype=torch.int64, device=dev)
        assert torch.equal(out[t0:t1, 0].to(torch.int64), t // n1), t0
        assert torch.equal(out[t0:t1, 1].to(torch.int64), t % n1), t0
    print("\n# %d tuples checked" % cnt, flush=True)


def test_count_near_ten_to_the_12():
    n0, n1, n2 = 100_003, 1_009, 10_007
    q = W.Query("chain3", [W.Relation("R0", [np.full(n0, 1, np.int32)]),
                           W.Relation("R1", [np.full(n1, 1, np.int32), np.full(n1, 2, np.int32)]),
                           W.Relation("R2", [np.full(n2, 2, np.int32)])],
                [(0, 0, 1, 0), (1, 1, 2, 0)], 0)
    plan = make_plan(q, **OPTS)
    plan.build_filters()
    plan.sieve()
    want = oracle.join_tree_dp(q)
    assert want[0] == n0 * n1 * n2
    assert plan.join() == want
    plan.build_filters()
    plan.sieve()
    plan.join_async()
    assert plan.join_wait() == (want[0], want[1], sj.SJ_OK)
