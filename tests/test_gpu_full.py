"""Full-size parity on the 4-way Zipf chain (4 x 10M rows) in the timed launch setup.

The plan uses the options the benchmark times (8 bits per key, k = 6, 512-bit
blocks, both passes) and replays its launch graphs. Survivor lists, every filter's
words, count and checksum are compared with the oracle exactly; the result tuples
are compared row by row with the oracle's sorted result (for a chain listed root
first the plan's enumeration order is relation-index order).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from sjtest import check_sieve, make_plan

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SEED = 0x5EED0002
OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=SEED)


@pytest.fixture(scope="module")
def chain4():
    return W.config2(seed=SEED, scale=1.0)


def test_chain4_full_size(chain4):
    q = chain4
    plan = make_plan(q, **OPTS)
    ref, rcnt, rchk = oracle.hash_join(q)
    for it in range(2):      # first call records the graphs, second replays them
        plan.build_filters()
        plan.sieve()
        check_sieve(q, plan, **OPTS)
        cnt, chk = plan.join()
        assert (cnt, chk) == (rcnt, rchk)
        out = plan.result()
        torch.cuda.synchronize()
        tup = out.cpu().numpy().astype(np.uint32)
        assert tup.shape == ref.shape
        assert np.array_equal(tup, ref), "tuples differ at call %d" % it
