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


def test_star_full_size():
    """Star: 100M-row fact table with four foreign keys, four 1M-row dimensions keeping
    10%: survivors, filters, count, checksum and tuples equal the oracle's."""
    q = W.config3(scale=1.0)
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=0x5EED0003)
    plan = make_plan(q, **opts)
    plan.build_filters()
    plan.sieve()
    check_sieve(q, plan, **opts)
    cnt, chk = plan.join()
    ref, rcnt, rchk = oracle.hash_join(q)
    assert (cnt, chk) == (rcnt, rchk)
    tup = plan.result().cpu().numpy().astype(np.uint32)
    assert np.array_equal(tup, ref)


def _check_triangle_tuples(q, tup, count, checksum):
    """Every tuple is a directed 3-cycle e1 = (a->b), e2 = (b->c), e3 = (c->a), and the
    tuples' count and checksum (oracle.checksum_of) are the oracle's (the intersection
    walk writes them in walk order; a missing, repeated or wrong tuple changes the
    checksum)."""
    src, dst = (torch.from_numpy(c).cuda() for c in q.rels[0].cols)
    t = tup.long()
    assert t.shape[0] == count
    assert torch.equal(dst[t[:, 0]], src[t[:, 1]])
    assert torch.equal(dst[t[:, 1]], src[t[:, 2]])
    assert torch.equal(dst[t[:, 2]], src[t[:, 0]])
    assert oracle.checksum_of(tup.cpu().numpy().astype(np.uint32)) == checksum


def test_triangle_one_64th():
    """The triangle workload at 1/64 scale (781,250 edges, 10.7M result tuples): count
    and checksum equal the oracle's adjacency-intersection count; every tuple is valid."""
    q = W.config4(scale=1 / 64)
    rc, rk = oracle.triangle_cycles(*q.rels[0].cols)
    plan = make_plan(q, bits_per_key=8, k=6, block_bits=512, passes=2, seed=0x5EED0004)
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    assert (cnt, chk) == (rc, rk)
    assert cnt % 3 == 0
    _check_triangle_tuples(q, plan.result(), cnt, chk)


def test_triangle_one_16th_golden():
    """1/16 scale (3.1M edges, 57M result tuples): count and checksum equal the stored
    oracle values (tests/golden/triangle_cycles.json)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "triangle_cycles.json")))
    case = next(c for c in g["cases"] if abs(c["scale"] - 1 / 16) < 1e-12)
    q = W.config4(scale=case["scale"])
    assert q.rels[0].nrows == case["edges"]
    plan = make_plan(q, bits_per_key=8, k=6, block_bits=512, passes=2, seed=0x5EED0004)
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    assert (cnt, chk) == (case["count"], case["checksum"])
    _check_triangle_tuples(q, plan.result(), cnt, chk)


def _golden_cases(min_scale):
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "triangle_cycles.json")))
    return [pytest.param(c, id="scale-%g" % c["scale"]) for c in g["cases"] if c["scale"] >= min_scale]


@pytest.mark.parametrize("case", _golden_cases(0.25))
def test_triangle_count_at_large_scale_golden(case):
    """The triangle workload at 1/4 size and above (generated on the GPU, identical to
    the numpy generator's edges): the intersection count and checksum equal the
    stored oracle values (tests/golden/triangle_cycles.json)."""
    q = W.config4(scale=case["scale"], device="cuda:0")
    assert q.rels[0].nrows == case["edges"]
    plan = make_plan(q, bits_per_key=8, k=6, block_bits=512, passes=2, seed=0x5EED0004)
    plan.build_filters()
    plan.sieve()
    assert plan.join() == (case["count"], case["checksum"])


def test_psyn_full_size():
    """The paper's synthetic join at its comparison sizes (Section 3.1.1: M = 10^7,
    r = 10^4, d = 10; 2e8 input rows). Count equals the closed form r * d^3 = 10^7, count
    and checksum equal the oracle's join-tree DP (stored by tests/golden/make_psyn_golden.py),
    and every one of the 10^7 tuples is checked: its three rows hold the same value, and
    the tuples are strictly increasing (so distinct). Valid, distinct and as many as the
    exact count, the tuples are exactly the result."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "psyn_full.json")))
    q = W.psyn(g["M"], g["r"], g["d"], seed=g["seed"])
    assert [r.nrows for r in q.rels] == g["rows"]
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=g["seed"])
    plan = make_plan(q, **opts)
    for _ in range(2):
        plan.build_filters()
        surv = plan.sieve(survivors=True)
        cnt, chk = plan.join()
        assert cnt == g["r"] * g["d"] ** 3 == g["count"]
        assert chk == g["checksum"]
        # no false negatives: the r shared values survive with their d rows each
        assert all(s >= g["r"] * g["d"] for s in surv), surv
    tup = plan.result()
    vals = [plan.rels[i].cols[0][tup[:, i].long()] for i in range(3)]
    assert bool(torch.equal(vals[0], vals[1])) and bool(torch.equal(vals[1], vals[2]))
    t = tup.long()
    d = t[1:] - t[:-1]
    first = torch.where(d[:, 0] != 0, d[:, 0], torch.where(d[:, 1] != 0, d[:, 1], d[:, 2]))
    assert bool((first > 0).all()), "tuples are not strictly increasing"
