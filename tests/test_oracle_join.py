"""Pins of the oracle's join result (CPU only).

The oracle's binary hash join is checked against things that do not share its
code: a nested-loop brute force written here in pure Python, the join-tree DP
(numpy), the paper's worked example (the synthetic benchmark's r*d^3 count),
closed forms for star joins and two-relation joins, and an adjacency-intersection
triangle count.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

M64 = (1 << 64) - 1


def py_mix64(z):
    # SplitMix64 output function, written out again in plain Python integers
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def brute_force(q):
    """Nested loops over the relations in index order; an edge is checked once both ends are bound."""
    n = len(q.rels)
    elig = []
    for rel in q.rels:
        rows = []
        for r in range(rel.nrows):
            if rel.pred is None or rel.pred[1] <= int(rel.cols[rel.pred[0]][r]) < rel.pred[2]:
                rows.append(r)
        elig.append(rows)
    checks = [[] for _ in range(n)]
    for (a, ca, b, cb) in q.edges:
        checks[max(a, b)].append((a, ca, b, cb))
    out = []
    cur = [0] * n

    def rec(i):
        if i == n:
            out.append(tuple(cur))
            return
        for r in elig[i]:
            cur[i] = r
            if all(int(q.rels[a].cols[ca][cur[a]]) == int(q.rels[b].cols[cb][cur[b]])
                   for (a, ca, b, cb) in checks[i]):
                rec(i + 1)

    rec(0)
    out.sort()
    chk = 0
    for t in out:
        f = 1
        for i, rid in enumerate(t):
            f = (f * (py_mix64((i << 32) | rid) | 1)) & M64
        chk = (chk + f) & M64
    return out, chk


def test_mixer_published_vectors():
    # MurmurHash3_x86_32 of the empty input is fmix32(seed): published vectors for seeds 1, 2^32-1
    assert oracle.fmix32(1) == 0x514E28B7
    assert oracle.fmix32(0xFFFFFFFF) == 0x81F16F39
    assert oracle.fmix32(0) == 0
    # SplitMix64 seeded with 0: first output is mix64(0x9E3779B97F4A7C15)
    assert oracle.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    rng = np.random.default_rng(5)
    z = rng.integers(0, 2**63, size=1000, dtype=np.int64).astype(np.uint64) * np.uint64(3)
    got = oracle.mix64_np(z)
    for a, b in zip(z[:50], got[:50]):
        assert int(b) == py_mix64(int(a)) == oracle.mix64(int(a))


@pytest.mark.parametrize("seed", range(400))
def test_hash_join_equals_brute_force(seed):
    q = W.tiny_random(seed)
    tup, cnt, chk = oracle.hash_join(q)
    bf, bchk = brute_force(q)
    assert cnt == len(bf)
    assert [tuple(int(x) for x in t) for t in tup] == bf
    assert chk == bchk


@pytest.mark.parametrize("seed", range(60))
def test_hash_join_root_invariant(seed):
    q = W.tiny_random(1000 + seed)
    base = oracle.hash_join(q)
    for root in range(len(q.rels)):
        tup, cnt, chk = oracle.hash_join(q, root=root)
        assert cnt == base[1] and chk == base[2]
        assert np.array_equal(tup, base[0])


@pytest.mark.parametrize("seed", range(150))
def test_dp_equals_brute_force_acyclic(seed):
    q = W.tiny_random(2000 + seed, kind=["chain", "star", "tree", "pair"][seed % 4])
    bf, bchk = brute_force(q)
    for root in range(len(q.rels)):
        assert oracle.join_tree_dp(q, root=root) == (len(bf), bchk)


def _psyn_cases():
    path = os.path.join(os.path.dirname(__file__), "golden", "psyn_counts.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(tuple(int(x) for x in line.split()))
    return rows


@pytest.mark.parametrize("M,r,d,expected", _psyn_cases())
def test_psyn_count_matches_paper(M, r, d, expected):
    q = W.psyn(M, r, d, seed=11)
    assert oracle.join_tree_dp(q)[0] == expected
    if expected <= 20000:
        tup, cnt, chk = oracle.hash_join(q)
        assert cnt == expected
        assert oracle.join_tree_dp(q)[1] == chk
        # every result row carries one of the r shared values
        vals = q.rels[0].cols[0][tup[:, 0]]
        assert len(np.unique(vals)) == r


def test_psyn_unsieved_intermediate():
    # without sieving, R join S alone has ((M + r) / 2) * d^2 tuples
    M, r, d = 2000, 100, 3
    q = W.psyn(M, r, d, seed=3)
    q2 = W.Query("rs", q.rels[:2], [q.edges[0]])
    assert oracle.join_tree_dp(q2)[0] == ((M + r) // 2) * d * d


def test_config1_hash_join_equals_dp():
    q = W.config1(scale=0.3)
    tup, cnt, chk = oracle.hash_join(q)
    assert (cnt, chk) == oracle.join_tree_dp(q)
    assert oracle.checksum_of(tup) == chk
    # sorted, strictly increasing (no duplicate rid tuples)
    if cnt > 1:
        d = np.diff(tup.astype(np.int64), axis=0)
        first = np.argmax(d != 0, axis=1)
        assert np.all(d[np.arange(d.shape[0]), first] > 0)


def test_star_closed_form():
    q = W.star(200_000, 4, 5_000, 0.1, seed=7)
    # dimension keys are unique: a fact row joins iff every referenced dim row passes
    ok = np.ones(q.rels[0].nrows, dtype=bool)
    for i in range(4):
        dim = q.rels[i + 1]
        passing = np.zeros(5_000, dtype=bool)
        passing[dim.cols[0][dim.cols[1] < 500]] = True
        ok &= passing[q.rels[0].cols[i]]
    tup, cnt, chk = oracle.hash_join(q)
    assert cnt == int(ok.sum())
    assert np.array_equal(tup[:, 0], np.nonzero(ok)[0].astype(np.uint32))
    assert oracle.join_tree_dp(q) == (cnt, chk)


def test_two_relation_count():
    # Bloomjoin's setting (Section 2.1): |R join S| = sum_k f_R(k) f_S(k)
    rng = np.random.default_rng(1)
    a = rng.integers(-50, 50, size=3000).astype(np.int32)
    b = rng.integers(-60, 40, size=2000).astype(np.int32)
    q = W.Query("pair", [W.Relation("R", [a]), W.Relation("S", [b])], [(0, 0, 1, 0)])
    ka, ca = np.unique(a, return_counts=True)
    kb, cb = np.unique(b, return_counts=True)
    common, ia, ib = np.intersect1d(ka, kb, return_indices=True)
    expected = int(np.sum(ca[ia].astype(np.int64) * cb[ib]))
    assert oracle.hash_join(q)[1] == expected


def test_triangle_against_adjacency_intersection():
    q = W.triangle(6000, 1500, 2.1, seed=9)
    src, dst = q.rels[0].cols
    out = {}
    inn = {}
    for s, d in zip(src.tolist(), dst.tolist()):
        out.setdefault(s, set()).add(d)
        inn.setdefault(d, set()).add(s)
    # tuples (e1, e2, e3) = (a->b, b->c, c->a): for each edge a->b, |out(b) & in(a)|
    expected = sum(len(out.get(b, set()) & inn.get(a, set())) for a, b in zip(src.tolist(), dst.tolist()))
    tup, cnt, chk = oracle.hash_join(q)
    assert cnt == expected
    assert cnt % 3 == 0          # closed under rotation of the three edges
    rot = tup[:, [1, 2, 0]]
    rot = rot[np.lexsort((rot[:, 2], rot[:, 1], rot[:, 0]))]
    assert np.array_equal(rot, tup)


def test_edge_cases_empty_and_extremes():
    e = np.zeros(0, dtype=np.int32)
    x = np.array([-2**31, 2**31 - 1, -2**31, 0], dtype=np.int32)
    q = W.Query("e", [W.Relation("R", [x]), W.Relation("S", [e])], [(0, 0, 1, 0)])
    assert oracle.hash_join(q)[1] == 0
    q = W.Query("x", [W.Relation("R", [x]), W.Relation("S", [x.copy()])], [(0, 0, 1, 0)])
    tup, cnt, chk = oracle.hash_join(q)
    assert cnt == 2 * 2 + 1 + 1
    assert (cnt, chk) == oracle.join_tree_dp(q)


@pytest.mark.parametrize("seed", range(12))
def test_triangle_cycles_matches_hash_join(seed):
    """The adjacency-intersection count agrees with the binary join plan and with
    brute force, on graphs with parallel edges, self-loops and negative vertex ids."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(1, 60))
    v = int(rng.integers(1, 9))
    src = (rng.integers(0, v, n) - (v // 2 if seed % 3 == 0 else 0)).astype(np.int32)
    dst = (rng.integers(0, v, n) - (v // 2 if seed % 3 == 0 else 0)).astype(np.int32)
    if seed % 4 == 1:
        src[:3] = dst[:3]                     # self-loops
    q = W.Query("tri", [W.Relation("E%d" % i, [src, dst]) for i in range(3)],
                [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 0, 0)])
    tup, cnt, chk = oracle.hash_join(q)
    bf = [(i, j, k) for i in range(n) for j in range(n) for k in range(n)
          if dst[i] == src[j] and dst[j] == src[k] and dst[k] == src[i]]
    assert cnt == len(bf)
    assert oracle.triangle_cycles(src, dst) == (cnt, chk)


def test_triangle_cycles_generated_graph():
    q = W.triangle(6000, 1500, 2.1, seed=9)
    src, dst = q.rels[0].cols
    tup, cnt, chk = oracle.hash_join(q)
    assert oracle.triangle_cycles(src, dst) == (cnt, chk)


@pytest.mark.parametrize("seed", range(8))
def test_triangle_cycles_with_a_subset_as_first_relation(seed):
    """E1 a subset of the rows (renumbered 0..m-1), E2 = E3 the whole list: equal to the
    binary join plan on that query and to brute force; the subset of all rows in order
    is the plain call."""
    rng = np.random.default_rng(1700 + seed)
    n = int(rng.integers(1, 70))
    v = int(rng.integers(1, 8))
    src = (rng.integers(0, v, n) - (3 if seed % 2 else 0)).astype(np.int32)
    dst = (rng.integers(0, v, n) - (3 if seed % 2 else 0)).astype(np.int32)
    idx = np.sort(rng.choice(n, int(rng.integers(0, n + 1)), replace=False))
    s1, d1 = src[idx], dst[idx]
    q = W.Query("sub", [W.Relation("S", [s1, d1]), W.Relation("E2", [src, dst]), W.Relation("E3", [src, dst])],
                [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 0, 0)])
    _, cnt, chk = oracle.hash_join(q)
    bf = [(i, j, k) for i in range(len(idx)) for j in range(n) for k in range(n)
          if d1[i] == src[j] and dst[j] == src[k] and dst[k] == s1[i]]
    assert cnt == len(bf)
    assert oracle.triangle_cycles(src, dst, e1=(s1, d1)) == (cnt, chk)
    assert oracle.triangle_cycles(src, dst, e1=(src, dst)) == oracle.triangle_cycles(src, dst)
