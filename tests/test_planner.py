"""The planner's estimates (Section 2.1, Eq. (1)-(3) as read in paper_2308_16370_amd.planner)
against what the sieve really keeps, computed by the oracle (oracle.sieve, exact survivor
lists of the plan's schedule) on inputs where the planner's assumptions hold (keys
spread uniformly over their ranges, independent columns): uniform chains, the paper's
synthetic join, a star, and a two-relation Bloomjoin. Skewed (Zipf) keys break the
uniformity assumption; there the estimate is only reported, not pinned.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2308_16370_amd import planner as P

SEED32 = oracle.filter_seed(1)


@pytest.mark.parametrize("n,bpk,k,B", [(100_000, 8, 6, 512), (50_000, 4, 2, 512), (80_000, 10, 7, 256)])
def test_fpr_matches_a_built_filter(n, bpk, k, B):
    """fpr(D, nblocks, k, B) against the measured false-positive rate of the oracle's filter."""
    rng = np.random.default_rng(n + k)
    keys = rng.choice(1 << 30, size=n + 1_000_000, replace=False).astype(np.int32)
    ins, q = keys[:n], keys[n:]
    nb = oracle.bf_nblocks(n, bpk, B)
    w = oracle.bf_build(ins, None, nb, k, B, SEED32)
    rate = float(oracle.bf_probe(w, q, None, nb, k, B, SEED32).mean())
    est = P.fpr(n, nb, k, B)
    sig = math.sqrt(est * (1 - est) / q.shape[0])
    assert abs(rate - est) <= 0.06 * est + 5 * sig


def test_bloomjoin_cardinality_two_relations():
    """n = 2 is Bloomjoin: T's rows that pass S's filter are the matching ones plus the
    false positives (Eq. (1) read as a tuple count)."""
    q = W.chain(2, [60_000, 200_000], 150_000, 0.0, 0x5EED0B01)
    st = P.column_stats(q)
    S, _ = oracle.sieve(q, bits_per_key=2, k=2, block_bits=512, passes=1, seed=1, root=0)
    e = P.estimate(st, q.edges, 0, bits_per_key=2, k=2, block_bits=512, passes=1)
    assert abs(e.survivors[0] / len(S[0]) - 1) < 0.05
    # the same with the matching fraction and the false positives taken from the data
    left = q.rels[0].cols[1]
    right_keys = np.unique(q.rels[1].cols[0])
    sc = int(np.isin(left, right_keys).sum())
    nb = oracle.bf_nblocks(q.rels[1].nrows, 2, 512)
    bc = P.bloomjoin_cardinality(left.shape[0], sc, right_keys.shape[0], nb, 2, 512)
    assert abs(bc / len(S[0]) - 1) < 0.01


@pytest.mark.parametrize("name", ["config1", "chain4_uniform", "psyn", "star", "config1_bpk2"])
@pytest.mark.parametrize("passes", [1, 2])
def test_estimates_follow_the_sieve(name, passes):
    q, opts = {
        "config1": (W.config1(), dict(bits_per_key=10, k=7)),
        "chain4_uniform": (W.chain(4, 50_000, 40_000, 0.0, 3), dict(bits_per_key=8, k=6)),
        "psyn": (W.psyn(20_000, 100, 5, seed=2), dict(bits_per_key=8, k=6)),
        "star": (W.star(200_000, 4, 20_000, 0.1, 5), dict(bits_per_key=8, k=6)),
        "config1_bpk2": (W.config1(), dict(bits_per_key=2, k=2)),
    }[name]
    st = P.column_stats(q)
    e = P.estimate(st, q.edges, 0, passes=passes, block_bits=512, **opts)
    S, _ = oracle.sieve(q, passes=passes, root=0, block_bits=512, seed=1, **opts)
    for j, (est, got) in enumerate(zip(e.survivors, (len(s) for s in S))):
        assert 0.7 * got - 5 <= est <= 1.4 * got + 5, (j, est, got)


def test_choose_returns_the_cheapest_candidate():
    q = W.config1(scale=0.3)
    st = P.column_stats(q)
    best = P.choose(st, q.edges, 0)
    for b in (4, 8, 16):
        for p in (1, 2):
            assert best.bytes <= P.estimate(st, q.edges, 0, b, 6, 512, p).bytes
    assert best.bits_per_key in (4, 6, 8, 12, 16) and best.passes in (1, 2) and best.k in (2, 4, 6)
