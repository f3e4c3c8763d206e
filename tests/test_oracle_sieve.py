"""Pins of the oracle's pruning phase (CPU only).

* Soundness: a filter has no false negatives, so every row that takes part in a
  result survives every pass (the sieve only removes rows that cannot join).
* With exact key sets in place of Bloom filters the backward pass is a semijoin
  program toward the root (the root becomes fully reduced) and the added forward
  pass completes the full reducer of an acyclic join: every relation is then exactly
  its projection of the result.
* A second pass never keeps a row the first pass dropped.
* The "stop early" property: over fully reduced relations every prefix of the
  left-deep plan extends to a result, so no intermediate exceeds the result size.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def projections(q, tup):
    return [np.unique(tup[:, i]).astype(np.uint32) for i in range(len(q.rels))]


@pytest.mark.parametrize("seed", range(200))
def test_sieve_sound_bloom(seed):
    q = W.tiny_random(3000 + seed)
    tup, cnt, _ = oracle.hash_join(q)
    proj = projections(q, tup)
    for passes in (1, 2):
        S, _ = oracle.sieve(q, bits_per_key=4, k=3, passes=passes, seed=seed)
        for i in range(len(q.rels)):
            assert np.all(np.isin(proj[i], S[i]))
            assert np.all(np.diff(S[i].astype(np.int64)) > 0)


@pytest.mark.parametrize("seed", range(200))
def test_exact_sieve_is_full_reducer(seed):
    q = W.tiny_random(4000 + seed, kind=["chain", "star", "tree", "pair"][seed % 4])
    tup, cnt, _ = oracle.hash_join(q)
    proj = projections(q, tup)
    S2, _ = oracle.sieve(q, passes=2, exact=True)
    for i in range(len(q.rels)):
        assert np.array_equal(S2[i], proj[i])
    S1, _ = oracle.sieve(q, passes=1, exact=True)
    assert np.array_equal(S1[q.root], proj[q.root])
    for i in range(len(q.rels)):
        assert np.all(np.isin(S2[i], S1[i]))


@pytest.mark.parametrize("seed", range(80))
def test_cyclic_exact_sieve_sound(seed):
    q = W.tiny_random(5000 + seed, kind=["triangle", "cycle4", "selfjoin"][seed % 3])
    tup, cnt, _ = oracle.hash_join(q)
    proj = projections(q, tup)
    for passes in (1, 2):
        S, _ = oracle.sieve(q, passes=passes, exact=True)
        for i in range(len(q.rels)):
            assert np.all(np.isin(proj[i], S[i]))


def test_second_pass_only_removes():
    q = W.config1(scale=0.2)
    S1, _ = oracle.sieve(q, 10, 7, 512, passes=1, seed=3)
    S2, _ = oracle.sieve(q, 10, 7, 512, passes=2, seed=3)
    for a, b in zip(S1, S2):
        assert np.all(np.isin(b, a))
    tup, cnt, chk = oracle.hash_join(q)
    # the join over the survivors alone gives the same result (no false negatives)
    assert oracle.join_tree_dp(q, sels=S2) == (cnt, chk)
    assert oracle.join_tree_dp(q, sels=S1) == (cnt, chk)


def test_stop_early_on_reduced_relations():
    q = W.config1(scale=0.2)
    S, _ = oracle.sieve(q, passes=2, exact=True)
    cnt = oracle.join_tree_dp(q)[0]
    # the k-relation prefix R1..Rk of the chain, over the reduced relations
    for k in range(2, len(q.rels) + 1):
        sub = W.Query("p", q.rels[:k], q.edges[:k - 1])
        assert oracle.join_tree_dp(sub, sels=S[:k])[0] <= cnt


def test_psyn_sieve_sizes():
    # P-syn: the sieved S and R keep r*d rows each (plus false positives) and T keeps r*d
    M, r, d = 20000, 100, 3
    q = W.psyn(M, r, d, seed=5)
    S, _ = oracle.sieve(q, passes=2, exact=True)
    assert [len(s) for s in S] == [r * d] * 3
    Sb, _ = oracle.sieve(q, bits_per_key=8, k=6, passes=2, seed=1)
    for s in Sb:
        assert r * d <= len(s) <= r * d + 0.1 * M * d
