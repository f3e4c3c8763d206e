"""Filter builds at the block counts where the build changes shape, against the oracle.

A filter of n keys has ceil(bits_per_key * n / B) blocks of B bits (Section 2.1). The
device picks the build's region size from that count: the largest power of two up to
16 KB of filter that still gives at least 256 regions, and never under 8 blocks. The
block counts below sit on each side of the points where that choice changes (8 blocks
per region up to 2047 blocks, then 16, 32, ... up to 16 KB regions from 65536 blocks on
for 512-bit blocks), plus a single block and a few blocks, for 256-, 512- and 1024-bit
blocks. The row counts are ragged (one below a multiple of the keys per block) as well
as exact. Keys are uniform 32-bit values with one heavy hitter that takes a quarter of
the rows, so tiles repeat keys and the build's duplicate filtering is exercised.

Each case is a two-relation join R0.c0 = R1.c0 with root R0: R1's backward filter has
the block count under test; R0's survivors build the forward filter that R1 is probed
with. Filter words and survivor lists must equal the oracle's bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from sjtest import check_sieve, make_plan

pytestmark = pytest.mark.gpu

BPK = 8
K = 6


def _cases():
    out = []
    for bb in (256, 512, 1024):
        kpb = bb // BPK   # keys per block at 8 bits per key
        region16k = 16384 * 8 // bb   # blocks in a 16 KB region
        for nb in (1, 3, 8, 9, 255, 256, 2047, 2048, 2049, 4095, 4096, 4097,
                   256 * region16k - 1, 256 * region16k, 256 * region16k + 1):
            for ragged in (False, True):
                if ragged and nb == 1:
                    continue
                n = nb * kpb - (kpb // 2 if ragged else 0)
                out.append(pytest.param(bb, nb, n, id="B%d-nb%d-%s" % (bb, nb, "ragged" if ragged else "exact")))
    return out


def _query(n1, seed):
    rng = np.random.default_rng(seed)
    r1 = rng.integers(-2**31, 2**31, size=n1, dtype=np.int64).astype(np.int32)
    hot = np.int32(rng.integers(-2**31, 2**31))
    r1[rng.random(n1) < 0.25] = hot
    n0 = 3000
    # R0: half its keys from R1 (not the heavy hitter, which would only inflate the
    # result), half random
    pick = r1[rng.integers(0, n1, size=n0)]
    r0 = np.where(rng.random(n0) < 0.5, pick, rng.integers(-2**31, 2**31, size=n0).astype(np.int32))
    r0[r0 == hot] = hot ^ np.int32(1)
    rels = [W.Relation("R0", [r0.astype(np.int32)]), W.Relation("R1", [r1])]
    return W.Query("pair", rels, [(0, 0, 1, 0)], 0)


@pytest.mark.parametrize("bb,nb,n", _cases())
def test_filter_build_at_region_thresholds(bb, nb, n):
    q = _query(n, 0x5EED0F00 + nb * 3 + bb)
    opts = dict(bits_per_key=BPK, k=K, block_bits=bb, passes=2, seed=0x5EED0F01)
    plan = make_plan(q, **opts)
    plan.build_filters()
    plan.sieve()
    S, F = check_sieve(q, plan, **opts)
    assert F[("bwd", 1)][1] == nb
    assert S[0].shape[0] > 0
