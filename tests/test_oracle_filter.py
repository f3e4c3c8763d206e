"""Pins of the oracle's blocked Bloom filter (CPU only).

The filter is checked against probability laws rather than against its own code:
no false negatives (Bloom's defining property), the expected number of set bits
(the paper's Eq. (3) for the bits set in a filter, generalised to k hashes), the
false-positive rate predicted from the filter's own per-block fill, the blocked
filter's false-positive law, and uniformity of the block and bit choice.
"""
import math

import numpy as np
import pytest
from scipy.stats import binom, chi2

import oracle

SEED32 = oracle.filter_seed(0x5EED)


def _keys(rng, n, q):
    k = rng.choice(2**32, size=n + q, replace=False).astype(np.int64) - 2**31
    return k[:n].astype(np.int32), k[n:].astype(np.int32)


def _popcounts(words, B):
    per = np.unpackbits(words.view(np.uint8)).reshape(-1, B).sum(axis=1)
    return per


def test_nblocks_is_ceiling():
    assert oracle.bf_nblocks(100_000, 10, 512) == math.ceil(1_000_000 / 512) == 1954
    assert oracle.bf_nblocks(10_000_000, 8, 512) == 156_250
    assert oracle.bf_nblocks(0, 8, 512) == 1
    assert oracle.bf_nblocks(1, 8, 1024) == 1
    assert oracle.bf_nblocks(65, 8, 256) == 3


@pytest.mark.parametrize("B", [256, 512, 1024])
def test_single_key_sets_bits_in_one_block(B):
    rng = np.random.default_rng(B)
    nb = 977
    for key in rng.integers(-2**31, 2**31, size=200):
        b, pos = oracle.bf_pattern(int(key), nb, 7, B, SEED32)
        w = oracle.bf_build(np.array([key], np.int32), None, nb, 7, B, SEED32)
        per = _popcounts(w, B)
        assert 0 <= b < nb and per[b] == len(set(pos)) and per.sum() == per[b]
        bits = np.unpackbits(w.view(np.uint8), bitorder="little").reshape(-1, B)[b]
        assert sorted(np.nonzero(bits)[0].tolist()) == sorted(set(pos))


@pytest.mark.parametrize("n,bpk,k,B", [(50_000, 8, 6, 512), (20_000, 10, 7, 512), (30_000, 4, 2, 256),
                                       (30_000, 12, 12, 1024), (1, 8, 6, 512)])
def test_no_false_negatives(n, bpk, k, B):
    rng = np.random.default_rng(n + k)
    ins, _ = _keys(rng, n, 0)
    nb = oracle.bf_nblocks(n, bpk, B)
    w = oracle.bf_build(ins, None, nb, k, B, SEED32)
    assert oracle.bf_probe(w, ins, None, nb, k, B, SEED32).all()
    # row-selected build: exactly the selected keys are guaranteed present
    rows = np.sort(rng.choice(n, size=max(1, n // 3), replace=False)).astype(np.uint32)
    w2 = oracle.bf_build(ins, rows, nb, k, B, SEED32)
    assert oracle.bf_probe(w2, ins, rows, nb, k, B, SEED32).all()
    assert np.array_equal(w2 | w, w)


@pytest.mark.parametrize("n,bpk,k,B", [(200_000, 8, 6, 512), (100_000, 10, 7, 512), (100_000, 8, 6, 256),
                                       (100_000, 8, 6, 1024), (60_000, 1, 1, 512)])
def test_popcount_generalised_eq3(n, bpk, k, B):
    rng = np.random.default_rng(7 * n + k)
    ins, _ = _keys(rng, n, 0)
    nb = oracle.bf_nblocks(n, bpk, B)
    m = nb * B
    ones = int(_popcounts(oracle.bf_build(ins, None, nb, k, B, SEED32), B).sum())
    # Eq. (3): bits_S = F (1 - e^{-D_S / F}) for one hash; with k hashes F (1 - e^{-k D / F})
    eq3 = m * (1 - math.exp(-k * n / m))
    assert abs(ones - eq3) <= 0.01 * eq3
    # exact expectation for k independent uniform bits inside a Binomial(n, 1/nb)-loaded block
    z = (1 - 1 / B) ** k
    exact = m * (1 - (1 - (1 - z) / nb) ** n)
    assert abs(ones - exact) <= 5 * math.sqrt(exact * (1 - exact / m)) + 1


@pytest.mark.parametrize("n,bpk,k,B", [(200_000, 8, 6, 512), (100_000, 10, 7, 512), (100_000, 8, 6, 256),
                                       (100_000, 8, 6, 1024), (50_000, 4, 3, 512)])
def test_false_positive_rate(n, bpk, k, B):
    rng = np.random.default_rng(11 * n + k + B)
    Q = 2_000_000
    ins, qk = _keys(rng, n, Q)
    nb = oracle.bf_nblocks(n, bpk, B)
    m = nb * B
    w = oracle.bf_build(ins, None, nb, k, B, SEED32)
    fp = int(oracle.bf_probe(w, qk, None, nb, k, B, SEED32).sum())
    rate = fp / Q
    # (a) given the filter, a key that was not inserted hits a uniform block and k uniform
    #     bits in it: P = mean_b (X_b / B)^k with X_b the block's popcount -- exact
    cond = float(np.mean((_popcounts(w, B) / B) ** k))
    sig = math.sqrt(cond * (1 - cond) / Q)
    assert abs(rate - cond) <= 5 * sig
    # (b) the blocked-filter law: Binomial block loads, k independent bits per key
    i = np.arange(0, n + 1)
    pmf = binom.pmf(i, n, 1.0 / nb)
    law = float(np.sum(pmf * (1 - (1 - 1 / B) ** (k * i)) ** k))
    assert abs(rate - law) <= 0.06 * law + 5 * sig
    # (c) the textbook un-blocked rate (1 - e^{-kn/m})^k is a lower bound for the blocked filter
    std = (1 - math.exp(-k * n / m)) ** k
    assert rate >= std - 5 * sig


def test_block_and_bit_choice_uniform():
    rng = np.random.default_rng(3)
    n, nb, k, B = 400_000, 1000, 6, 512
    keys = rng.integers(-2**31, 2**31, size=n).astype(np.int32)
    loads = np.zeros(nb, np.int64)
    posh = np.zeros(B, np.int64)
    for key in keys[:20000]:
        b, pos = oracle.bf_pattern(int(key), nb, k, B, SEED32)
        loads[b] += 1
        for p in pos:
            posh[p] += 1
    for h in (loads, posh):
        e = h.sum() / h.shape[0]
        stat = float(((h - e) ** 2 / e).sum())
        df = h.shape[0] - 1
        assert chi2.sf(stat, df) > 1e-6


def test_sequential_keys_spread():
    # structured keys (1..n, as in the paper's synthetic benchmark) still fill blocks evenly
    n, bpk, k, B = 100_000, 8, 6, 512
    keys = np.arange(1, n + 1, dtype=np.int32)
    nb = oracle.bf_nblocks(n, bpk, B)
    w = oracle.bf_build(keys, None, nb, k, B, SEED32)
    q = np.arange(n + 1, n + 1 + 1_000_000, dtype=np.int32)
    rate = oracle.bf_probe(w, q, None, nb, k, B, SEED32).mean()
    cond = float(np.mean((_popcounts(w, B) / B) ** k))
    assert abs(rate - cond) <= 5 * math.sqrt(cond / 1_000_000)


@pytest.mark.parametrize("seed", range(6))
def test_bf_insert_properties(seed):
    """Inserts into a built filter (Section 2.4), pinned against the plain build: into an
    empty filter they equal the build; A then B equals the build of A and B; every
    inserted key is found afterwards; keys already present change nothing and are
    reported contained."""
    rng = np.random.default_rng(300 + seed)
    k, B, seed32 = [(6, 512, 7), (3, 256, 99), (8, 1024, 12345)][seed % 3]
    nb = int(rng.integers(1, 40))
    a = rng.integers(-2**31, 2**31, int(rng.integers(0, 300)), dtype=np.int64).astype(np.int32)
    b = rng.integers(-50, 50, int(rng.integers(1, 300)), dtype=np.int64).astype(np.int32)
    empty = np.zeros(nb * B // 32, dtype=np.uint32)
    wa, ca = oracle.bf_insert(empty, a, nb, k, B, seed32)
    assert np.array_equal(wa, oracle.bf_build(a, None, nb, k, B, seed32))
    wab, cb = oracle.bf_insert(wa, b, nb, k, B, seed32)
    assert np.array_equal(wab, oracle.bf_build(np.concatenate([a, b]), None, nb, k, B, seed32))
    assert oracle.bf_probe(wab, np.concatenate([a, b]), None, nb, k, B, seed32).all()
    again, c2 = oracle.bf_insert(wab, a, nb, k, B, seed32)
    assert np.array_equal(again, wab) and c2.all()
    # a key reported missing sets at least one new bit when inserted alone; a key
    # reported contained sets none
    for key, was in list(zip(b, cb))[:40]:
        w1, _ = oracle.bf_insert(wa, np.array([key], dtype=np.int32), nb, k, B, seed32)
        assert np.array_equal(w1, wa) == bool(was)
