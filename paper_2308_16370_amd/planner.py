"""Planner estimates before a query runs: expected survivors of every sieve step and a
choice of bits per key and passes (arXiv 2308.16370, Section 2.1, Eq. (1)-(3)).

The paper gives the Bloomjoin cardinality of relation T probed by a filter on S as
Eq. (1), with the fraction alpha of non-matching T tuples (Eq. (2)) and the number of
set bits of S's filter (Eq. (3)). As printed, Eq. (1) adds a number of bits to a number
of tuples; it is read here as what it estimates: the T tuples that pass are the ones
that truly match (the semijoin cardinality SC_T) plus the non-matching ones that the
filter lets through, each with the filter's false-positive rate:

    BC_T = SC_T + (C_T - SC_T) * fpr

with Eq. (3) generalised to k bits per key and to cache-line-blocked filters: the
distinct keys D_S spread over the filter's blocks with Poisson loads, and a key that
was not inserted passes when all k of its bits (independent and uniform inside one
block of B bits) are set, so fpr = sum_i Pois(i; D_S / nblocks) (1 - (1 - 1/B)^(k i))^k.

The truly matching fraction needs the data; the planner takes per-column statistics
(row count after the predicate; per join column the distinct keys and their smallest
and largest value) and assumes that the distinct keys of a column are spread uniformly
over its value range, independently of other columns and relations: of D_T keys over a
range of width w_T, the ones that also occur among D_S keys over w_S number
|overlap of the ranges| * (D_T / w_T) * (D_S / w_S), and a row of T matches with the
fraction of its column's keys that do. A probe on a column keeps whole keys of that
column; a relation of C rows with D distinct keys on another column that keeps a
fraction f of its rows keeps D (1 - (1 - f)^(C / D)) of them. The schedule is the
plan's (backward pass from the leaves, root sieve, forward pass with passes = 2), and
filters are sized by the rows inserted (ceil(bits_per_key * n / B) blocks).

`choose` evaluates candidate (bits_per_key, passes) pairs with a byte model of the
sieve and the join (the kernels' algorithmic bytes) and returns the cheapest. It only
reads the statistics: a plan made with the chosen options returns the same result as
with any other options.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


def fpr(distinct: float, nblocks: int, k: int, block_bits: int) -> float:
    """Expected false-positive rate of a blocked filter of `nblocks` blocks holding
    `distinct` keys with k independent uniform bits per key inside its block."""
    if distinct <= 0:
        return 0.0
    lam = distinct / max(1, nblocks)
    hi = int(lam + 12 * math.sqrt(lam) + 40)
    i = np.arange(0, hi + 1, dtype=np.float64)
    # Poisson pmf in log space (stable for large loads)
    logp = i * math.log(lam) - lam - np.array([math.lgamma(x + 1) for x in i])
    pmf = np.exp(logp)
    return float(np.sum(pmf * (1.0 - (1.0 - 1.0 / block_bits) ** (k * i)) ** k))


def bloomjoin_cardinality(c_t: float, sc_t: float, distinct_s: float, nblocks: int, k: int,
                          block_bits: int) -> float:
    """Eq. (1) read as a tuple count: matching T tuples plus the non-matching ones the
    filter on S lets through."""
    return sc_t + (c_t - sc_t) * fpr(distinct_s, nblocks, k, block_bits)


def distinct_after(distinct: float, rows: float, keep: float) -> float:
    """Distinct keys left when a fraction `keep` of `rows` rows (independently) survives."""
    if rows <= 0 or distinct <= 0:
        return 0.0
    per = rows / distinct
    return distinct * (1.0 - (1.0 - min(1.0, max(0.0, keep))) ** per)


@dataclass
class RelStats:
    rows: int                                   # rows passing the relation's predicate
    distinct: Dict[int, int] = field(default_factory=dict)   # join column -> distinct keys (eligible rows)
    vrange: Dict[int, Tuple[int, int]] = field(default_factory=dict)   # join column -> (min, max) key


def match_fraction(d_t: float, r_t: Tuple[int, int], d_s: float, r_s: Tuple[int, int]) -> float:
    """Fraction of T's distinct keys that also occur among S's, with each side's keys
    spread uniformly over its value range."""
    if d_t <= 0 or d_s <= 0:
        return 0.0
    lo, hi = max(r_t[0], r_s[0]), min(r_t[1], r_s[1])
    if hi < lo:
        return 0.0
    w_t = r_t[1] - r_t[0] + 1.0
    w_s = r_s[1] - r_s[0] + 1.0
    shared = (hi - lo + 1.0) * (d_t / w_t) * min(1.0, d_s / w_s)
    return min(1.0, shared / d_t)


def column_stats(query) -> List[RelStats]:
    """Exact statistics of a workloads.Query's relations (host columns): eligible rows and
    distinct keys per join column."""
    out = []
    jcols = {}
    for a, ca, b, cb in query.edges:
        jcols.setdefault(a, set()).add(ca)
        jcols.setdefault(b, set()).add(cb)
    for r, rel in enumerate(query.rels):
        if rel.pred is None:
            sel = slice(None)
        else:
            c, lo, hi = rel.pred
            v = np.asarray(rel.cols[c])
            sel = (v >= lo) & (v < hi)
        st = RelStats(int(np.count_nonzero(sel)) if rel.pred is not None else rel.nrows)
        for c in sorted(jcols.get(r, ())):
            u = np.unique(np.asarray(rel.cols[c])[sel])
            st.distinct[c] = int(u.shape[0])
            st.vrange[c] = (int(u[0]), int(u[-1])) if u.shape[0] else (0, -1)
        out.append(st)
    return out


class _Tree:
    def __init__(self, n: int, edges: Sequence[Tuple[int, int, int, int]], root: int):
        adj = [[] for _ in range(n)]
        for (a, ca, b, cb) in edges:
            adj[a].append((b, ca, cb))
            adj[b].append((a, cb, ca))
        self.parent, self.pcol, self.mycol = [-1] * n, [-1] * n, [-1] * n
        self.children = [[] for _ in range(n)]
        seen = [False] * n
        seen[root] = True
        order = []

        def dfs(u):
            order.append(u)
            for v, cu, cv in adj[u]:
                if not seen[v]:
                    seen[v] = True
                    self.parent[v], self.pcol[v], self.mycol[v] = u, cu, cv
                    self.children[u].append(v)
                    dfs(v)

        dfs(root)
        self.preorder = order
        self.postorder = []

        def post(u):
            for c in self.children[u]:
                post(c)
            self.postorder.append(u)

        post(root)
        self.root = root


@dataclass
class Estimate:
    survivors: List[float]                 # expected final survivors per relation
    backward: List[float]                  # expected survivors after the backward pass
    filters: List[Tuple[str, int, float, int]]   # (kind, relation, keys inserted, blocks)
    bytes: float                           # modelled algorithmic bytes of sieve + join
    bits_per_key: int
    k: int
    block_bits: int
    passes: int


def estimate(stats: Sequence[RelStats], edges: Sequence[Tuple[int, int, int, int]], root: int = 0,
             bits_per_key: int = 8, k: int = 6, block_bits: int = 512, passes: int = 2) -> Estimate:
    """Expected survivors of every relation along the plan's sieve schedule (acyclic
    join graphs), and the modelled bytes of the sieve and the join.

    Survival is tracked per relation as a fraction of its rows and, per join column, as
    the distinct keys left: a probe on column c keeps whole keys of c (the ones that
    match, plus false positives) and rows of other columns independently of their keys.
    In the forward pass, the parent's final keys on the edge are (up to false positives)
    a subset of the child's keys it was probed with, so the child keeps the fraction of
    its keys that the parent still holds (plus false positives)."""
    n = len(stats)
    t = _Tree(n, edges, root)
    B = block_bits
    nblk = lambda r: max(1, math.ceil(bits_per_key * r / B))
    rows = [float(s.rows) for s in stats]
    cols = [sorted(s.distinct) for s in stats]

    def rng(r, col):
        return stats[r].vrange.get(col, (0, max(0, stats[r].rows - 1)))

    # state per relation: surviving rows, and per column the fraction of its distinct
    # keys kept by probes on that column (keyfrac) and the row fraction kept by probes
    # on other columns is folded in when the distinct keys are read (dist)
    surv = list(rows)
    keyfrac = [{c: 1.0 for c in cols[r]} for r in range(n)]
    rowfrac_by = [{c: 1.0 for c in cols[r]} for r in range(n)]   # row fraction from probes on column c

    def dist(r, c):
        """Distinct keys of column c among relation r's current survivors."""
        d = stats[r].distinct.get(c, stats[r].rows)
        other = 1.0
        for c2, f in rowfrac_by[r].items():
            if c2 != c:
                other *= f
        per = rows[r] / max(1.0, d)
        return d * keyfrac[r].get(c, 1.0) * (1.0 - (1.0 - min(1.0, other)) ** per)

    def probe(r, c, frac_keys, fp):
        """Relation r's rows probed on column c: matching keys keep `frac_keys` of the keys
        still held (plus false positives at rate fp)."""
        keep = frac_keys + (1.0 - frac_keys) * fp
        keyfrac[r][c] = keyfrac[r].get(c, 1.0) * keep
        rowfrac_by[r][c] = rowfrac_by[r].get(c, 1.0) * keep
        surv[r] = surv[r] * keep

    filters = []
    byt = 0.0
    for j in t.postorder:
        c_in = surv[j]
        for ch in t.children[j]:
            ds = dist(ch, t.mycol[ch])
            dt_all = stats[j].distinct.get(t.pcol[ch], stats[j].rows)
            m = match_fraction(dt_all, rng(j, t.pcol[ch]), ds, rng(ch, t.mycol[ch]))
            nb = nblk(surv[ch])
            probe(j, t.pcol[ch], m, fpr(ds, nb, k, B))
            byt += 4 * c_in + nb * B / 8                      # column scanned, filter read

        if t.children[j]:
            byt += surv[j] * 4 * 3                            # survivor list written
        if j != root:
            nb = nblk(surv[j])
            filters.append(("backward", j, surv[j], nb))
            byt += surv[j] * 4 * 2 + nb * B / 8                # keys staged, filter written
    backward = list(surv)
    if passes == 2:
        for x in t.preorder:
            if x == root:
                continue
            p = t.parent[x]
            ds = dist(p, t.pcol[x])
            # the parent's keys on this edge are (up to false positives) a subset of the keys
            # of x's backward survivors, which it was probed with
            ratio = ds / max(1e-9, dist(x, t.mycol[x]))
            nb = nblk(surv[p])
            filters.append(("forward", x, surv[p], nb))
            byt += surv[p] * 4 * 2 + nb * B / 8 + 4 * surv[x] + nb * B / 8
            probe(x, t.mycol[x], min(1.0, ratio), fpr(ds, nb, k, B))
            byt += surv[x] * 4 * 3
    # join: every non-root relation bucketed (three radix passes of 16 bytes per entry,
    # gather and directory), every relation weighed once
    for j in range(n):
        if j != root:
            byt += surv[j] * (16 * 3 + 8 * 3 + 4)
        byt += surv[j] * (4 + len(t.children[j]) * 40 + 16)
    return Estimate(surv, backward, filters, byt, bits_per_key, k, block_bits, passes)


def choose(stats: Sequence[RelStats], edges: Sequence[Tuple[int, int, int, int]], root: int = 0,
           bits_per_key=(4, 6, 8, 12, 16), ks=(2, 4, 6), passes=(1, 2), block_bits: int = 512) -> Estimate:
    """The candidate with the fewest modelled bytes."""
    best: Optional[Estimate] = None
    for b in bits_per_key:
        for k in ks:
            for p in passes:
                e = estimate(stats, edges, root, b, k, block_bits, p)
                if best is None or e.bytes < best.bytes:
                    best = e
    return best
