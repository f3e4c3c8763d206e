"""The 64-ary wave search of the materialisation kernel, modelled step by step on the CPU.

Each block of output finds the root entry of its first and last index with a search in
which the 64 lanes of a wave read 64 evenly spaced pivots per round and a ballot keeps
the part of the range that holds the answer. This model takes the same steps (the same
pivots, the same narrowing, the same final round over at most 64 entries) and is
checked against bisect_right: the first index in [lo, hi) whose prefix weight exceeds
x, or hi. Ranges of every size up to 140 and around 64^2, 64^3 and 10^6, with runs of
equal weights (zero-weight root entries) and x below, inside and above the weights.
Every pivot read must fall inside [lo, hi).
"""
import bisect
import random


def _first_set(m):
    return (m & -m).bit_length() - 1


def wave_upper_bound(a, lo, hi, x, reads):
    while hi - lo > 64:
        step = (hi - lo + 63) // 64
        m = 0
        for lane in range(64):
            idx = lo + lane * step
            if idx < hi:
                reads.append(idx)
            if idx >= hi or a[idx] > x:
                m |= 1 << lane
        f = _first_set(m) if m else 64
        if f == 0:
            return lo
        hi = min(hi, lo + f * step)
        lo = lo + (f - 1) * step + 1
    m = 0
    for lane in range(64):
        idx = lo + lane
        if idx < hi:
            reads.append(idx)
        if idx >= hi or a[idx] > x:
            m |= 1 << lane
    return lo + _first_set(m) if m else hi


def _weights(rng, n):
    out, v = [], 0
    for _ in range(n):
        v += rng.choice([0, 0, 1, 2, 5, 1000])
        out.append(v)
    return out


def test_wave_search_equals_binary_search():
    rng = random.Random(1)
    cases = 0
    for n in list(range(0, 140)) + [4095, 4096, 4097, 262143, 262145, 1000003]:
        for _ in range(3 if n < 5000 else 1):
            a = _weights(rng, n)
            top = a[-1] if a else 0
            xs = [-1, 0, top, top + 1] + [rng.randint(-1, top + 2) for _ in range(20 if n < 5000 else 4)]
            for lo in sorted({0, min(1, n), n // 3}):
                for hi in sorted({n, max(lo, n - 1), lo}):
                    for x in xs:
                        reads = []
                        got = wave_upper_bound(a, lo, hi, x, reads)
                        assert got == bisect.bisect_right(a, x, lo, hi), (n, lo, hi, x)
                        assert all(lo <= r < hi for r in reads)
                        cases += 1
    assert cases > 50000


def test_rounds_for_a_million_entries():
    a = list(range(1_000_003))
    reads = []
    assert wave_upper_bound(a, 0, len(a), 777_777, reads) == 777_778
    assert len(reads) <= 4 * 64   # three rounds of 64 pivots and the final round
