"""Seeded synthetic join workloads.

This module only draws inputs: integer key columns, selection predicates and the
join graph that connects them. It holds none of the join or filter arithmetic, so
that the GPU path and the CPU oracle can both consume the same inputs without
sharing any of the method's code.

Every generator is deterministic in its ``seed``: each (table, column) stream is
drawn from its own ``numpy`` PCG64 generator keyed by ``SeedSequence([seed, table,
column, purpose])``.

Workload shapes (the paper's own datasets are not available; these synthetic
shapes stand in for them):

* ``chain``      -- R1(a,b) join R2(b,c) join ... on the shared attribute, every
                   key column i.i.d. uniform or Zipf(s) over a domain of D keys, with
                   an independent random rank->key permutation per (table, column).
* ``star``       -- a fact table of foreign keys into dimension tables whose rows
                   are selected by a range predicate on a second attribute.
* ``triangle``   -- one directed edge relation E(src, dst) used three times,
                   E1.dst = E2.src, E2.dst = E3.src, E3.dst = E1.src.
* ``clique3`` / ``clique4`` -- one directed edge relation E(src, dst) used once per
                   pair of vertex variables (a -> b, a -> c, b -> c for 3-cliques; the
                   six pairs of a, b, c, d for 4-cliques): the clique queries of the
                   paper's vote-network experiment (Section 3.1.3).
* ``psyn``       -- the paper's controlled-intermediate benchmark (Section 3.1.1,
                   "Synthetic Workload"): unary R, S, T over overlapping integer
                   ranges, every value repeated d times.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Relation", "Query", "rng_for", "zipf_ranks", "chain", "star", "triangle",
    "psyn", "clique3", "clique4", "config1", "config2", "config3", "config4", "config6",
    "tiny_random",
]


@dataclass
class Relation:
    """A relation instance: int32 key columns plus an optional range predicate.

    ``pred`` is ``(col, lo, hi)`` and keeps rows with ``lo <= cols[col][row] < hi``.
    Several Relation objects may share the same column arrays (self-joins).
    """
    name: str
    cols: List[np.ndarray]
    pred: Optional[Tuple[int, int, int]] = None

    @property
    def nrows(self) -> int:
        return int(self.cols[0].shape[0]) if self.cols else 0


@dataclass
class Query:
    """A multi-way equi-join: relations and edges ``(rel_a, col_a, rel_b, col_b)``."""
    name: str
    rels: List[Relation]
    edges: List[Tuple[int, int, int, int]]
    root: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def input_tuples(self) -> int:
        return sum(r.nrows for r in self.rels)


def rng_for(seed: int, *stream: int) -> np.random.Generator:
    """An independent PCG64 stream for (seed, *stream)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed) & (2**63 - 1), *stream])))


@functools.lru_cache(maxsize=8)
def _zipf_cdf(domain: int, s: float) -> np.ndarray:
    w = np.arange(1, domain + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)          # fixed summation order
    cdf /= cdf[-1]
    return cdf


def zipf_ranks(rng: np.random.Generator, n: int, domain: int, s: float) -> np.ndarray:
    """0-based ranks with P(rank i) proportional to (i+1)^-s over i < domain (inverse CDF)."""
    if s == 0.0:
        return rng.integers(0, domain, size=n, dtype=np.int64)
    cdf = _zipf_cdf(domain, s)
    u = rng.random(n)
    r = np.searchsorted(cdf, u, side="right")
    np.minimum(r, domain - 1, out=r)
    return r


def _key_column(seed: int, table: int, col: int, n: int, domain: int, s: float,
                offset: int = 0) -> np.ndarray:
    rng = rng_for(seed, table, col, 0)
    ranks = zipf_ranks(rng, n, domain, s)
    if s == 0.0:
        keys = ranks
    else:
        perm = rng_for(seed, table, col, 1).permutation(domain)
        keys = perm[ranks]
    return (keys + offset).astype(np.int32)


def chain(nrels: int, rows, domain: int, s: float, seed: int, name: str = "chain",
          offset: int = 0) -> Query:
    """R1(c0,c1) join R2(c0,c1) join ... with R_t.c1 = R_{t+1}.c0.

    ``rows`` is an int or a per-table list. Each column is i.i.d. Zipf(s) over
    ``domain`` keys (s = 0: uniform), with its own random rank->key permutation,
    so heavy hitters of neighbouring tables do not line up.
    """
    if isinstance(rows, int):
        rows = [rows] * nrels
    rels = []
    for t in range(nrels):
        cols = [_key_column(seed, t, c, rows[t], domain, s, offset) for c in range(2)]
        rels.append(Relation(f"R{t + 1}", cols))
    edges = [(t, 1, t + 1, 0) for t in range(nrels - 1)]
    return Query(name, rels, edges, 0, dict(kind="chain", domain=domain, s=s, seed=seed))


def star(fact_rows: int, ndims: int, dim_rows: int, keep: float, seed: int,
         fk_s: float = 0.0, name: str = "star") -> Query:
    """Fact F(fk_1..fk_m) with fk_i over [0, dim_rows); dims D_i(pk, attr).

    ``pk`` and ``attr`` are independent random permutations of [0, dim_rows), and
    the predicate ``attr < keep * dim_rows`` keeps exactly that fraction of rows.
    Foreign keys are uniform (fk_s = 0) or Zipf(fk_s) over the dimension rows.
    """
    fcols = []
    for i in range(ndims):
        rng = rng_for(seed, 0, i, 0)
        if fk_s == 0.0:
            fcols.append(rng.integers(0, dim_rows, size=fact_rows, dtype=np.int32))
        else:
            r = zipf_ranks(rng, fact_rows, dim_rows, fk_s)
            fcols.append(rng_for(seed, 0, i, 1).permutation(dim_rows)[r].astype(np.int32))
    rels = [Relation("F", fcols)]
    cut = int(round(keep * dim_rows))
    for i in range(ndims):
        pk = rng_for(seed, i + 1, 0, 1).permutation(dim_rows).astype(np.int32)
        attr = rng_for(seed, i + 1, 1, 1).permutation(dim_rows).astype(np.int32)
        rels.append(Relation(f"D{i + 1}", [pk, attr], pred=(1, 0, cut)))
    edges = [(0, i, i + 1, 0) for i in range(ndims)]
    return Query(name, rels, edges, 0, dict(kind="star", keep=keep, seed=seed))


def powerlaw_edges(nedges: int, nverts: int, gamma: float, seed: int,
                   device: Optional[str] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Directed Chung-Lu edges: P(src = v), P(dst = v) proportional to (v+1)^(-1/(gamma-1)).

    Self-loops and repeated (src, dst) pairs are rejected; the first ``nedges``
    distinct pairs in draw order are kept, then vertex ids are randomly relabelled.
    With ``device`` (a torch device name) the searches and the de-duplication run in
    torch there; the random draws, the float64 CDF and every decision are the same,
    so the edges are identical to the numpy path's.
    """
    if device is not None:
        return _powerlaw_edges_torch(nedges, nverts, gamma, seed, device)
    w = (np.arange(1, nverts + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rng = rng_for(seed, 0, 0, 0)
    keys = np.empty(0, dtype=np.int64)
    order = np.empty(0, dtype=np.int64)
    drawn = 0
    batch = int(nedges * 1.3) + 1024
    while True:
        src = np.minimum(np.searchsorted(cdf, rng.random(batch), side="right"), nverts - 1)
        dst = np.minimum(np.searchsorted(cdf, rng.random(batch), side="right"), nverts - 1)
        k = src.astype(np.int64) * nverts + dst
        pos = np.arange(drawn, drawn + batch, dtype=np.int64)
        ok = src != dst
        keys = np.concatenate([keys, k[ok]])
        order = np.concatenate([order, pos[ok]])
        drawn += batch
        uk, first = np.unique(keys, return_index=True)
        if uk.shape[0] >= nedges:
            keep = np.sort(first)[:nedges]          # first occurrences in draw order
            sel = keys[keep]
            break
        keys, order = keys[np.sort(first)], order[np.sort(first)]
        batch = max(1024, int((nedges - uk.shape[0]) * 1.5))
    relabel = rng_for(seed, 0, 0, 1).permutation(nverts)
    s = relabel[sel // nverts].astype(np.int32)
    d = relabel[sel % nverts].astype(np.int32)
    return s, d


def _powerlaw_edges_torch(nedges, nverts, gamma, seed, device):
    import torch

    w = (np.arange(1, nverts + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf_t = torch.from_numpy(cdf).to(device)
    rng = rng_for(seed, 0, 0, 0)
    keys = torch.empty(0, dtype=torch.int64, device=device)
    drawn = 0
    batch = int(nedges * 1.3) + 1024
    while True:
        u_src = torch.from_numpy(rng.random(batch)).to(device)
        u_dst = torch.from_numpy(rng.random(batch)).to(device)
        src = torch.clamp(torch.searchsorted(cdf_t, u_src, right=True), max=nverts - 1)
        dst = torch.clamp(torch.searchsorted(cdf_t, u_dst, right=True), max=nverts - 1)
        del u_src, u_dst
        k = src * nverts + dst
        keys = torch.cat([keys, k[src != dst]])
        del src, dst, k
        drawn += batch
        # first occurrence of every distinct key, in draw order (a stable sort keeps
        # equal keys in draw order)
        sk, perm = torch.sort(keys, stable=True)
        head = torch.ones_like(sk, dtype=torch.bool)
        head[1:] = sk[1:] != sk[:-1]
        first = torch.sort(perm[head]).values
        del sk, perm, head
        if first.shape[0] >= nedges:
            sel = keys[first[:nedges]].cpu().numpy()
            break
        keys = keys[first]
        batch = max(1024, int((nedges - first.shape[0]) * 1.5))
    relabel = rng_for(seed, 0, 0, 1).permutation(nverts)
    s = relabel[sel // nverts].astype(np.int32)
    d = relabel[sel % nverts].astype(np.int32)
    return s, d


def triangle(nedges: int, nverts: int, gamma: float, seed: int, name: str = "triangle",
             device: Optional[str] = None) -> Query:
    """E1(a,b) join E2(b,c) join E3(c,a) over one edge relation (three instances)."""
    src, dst = powerlaw_edges(nedges, nverts, gamma, seed, device)
    rels = [Relation(f"E{i + 1}", [src, dst]) for i in range(3)]
    edges = [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 0, 0)]
    return Query(name, rels, edges, 0, dict(kind="triangle", nverts=nverts, gamma=gamma, seed=seed))



def clique3(src: np.ndarray, dst: np.ndarray, name: str = "clique3") -> Query:
    """E(a,b) join E(b,c) join E(a,c) over one edge list: relations AB, BC, AC with
    AB.dst = BC.src, BC.dst = AC.dst and AC.src = AB.src."""
    rels = [Relation(n, [src, dst]) for n in ("AB", "BC", "AC")]
    edges = [(0, 1, 1, 0), (1, 1, 2, 1), (2, 0, 0, 0)]
    return Query(name, rels, edges, 0, dict(kind="clique3"))


# relations AB, AC, AD, BC, BD, CD (column 0: the earlier vertex, column 1: the later);
# each vertex variable joins its three relations by two edges
CLIQUE4_EDGES = [(0, 0, 1, 0), (0, 0, 2, 0),      # a
                 (0, 1, 3, 0), (0, 1, 4, 0),      # b
                 (1, 1, 3, 1), (1, 1, 5, 0),      # c
                 (2, 1, 4, 1), (2, 1, 5, 1)]      # d


def clique4(src: np.ndarray, dst: np.ndarray, name: str = "clique4") -> Query:
    """The 4-clique query over one edge list: relations AB, AC, AD, BC, BD, CD, each
    the edge list (x -> y for the pair xy), joined on the shared vertex variables."""
    rels = [Relation(n, [src, dst]) for n in ("AB", "AC", "AD", "BC", "BD", "CD")]
    return Query(name, rels, list(CLIQUE4_EDGES), 0, dict(kind="clique4"))

def psyn(M: int, r: int, d: int, seed: int, name: str = "psyn") -> Query:
    """The paper's synthetic R join S join T (Section 3.1.1).

    R holds 1..M, S holds 1..(M+r)/2 and T holds (M-r)/2+1..M, each value d
    times, rows shuffled. With half-open bounds S and T share exactly r values, so
    the natural join has r*d^3 results (the paper's count). M + r must be even.
    """
    if (M + r) % 2:
        raise ValueError("M + r must be even")
    lo_t = (M - r) // 2 + 1
    hi_s = (M + r) // 2
    parts = [np.arange(1, M + 1), np.arange(1, hi_s + 1), np.arange(lo_t, M + 1)]
    rels = []
    for i, (nm, p) in enumerate(zip("RST", parts)):
        col = np.repeat(p.astype(np.int32), d)
        col = col[rng_for(seed, i, 0, 0).permutation(col.shape[0])]
        rels.append(Relation(nm, [col]))
    edges = [(0, 0, 1, 0), (1, 0, 2, 0)]
    return Query(name, rels, edges, 0, dict(kind="psyn", M=M, r=r, d=d, seed=seed))


# ---- the named workload configurations ---------------------------------------------------

def config1(seed: int = 0x5EED0001, scale: float = 1.0) -> Query:
    """3-way chain, 100k rows per table, int32 keys uniform over [0, 50000)."""
    return chain(3, max(1, int(100_000 * scale)), 50_000, 0.0, seed, name="chain3_uniform")


def config2(seed: int = 0x5EED0002, scale: float = 1.0) -> Query:
    """4-way chain, 10M rows per table, Zipf(1.1) over 2^22 keys, permuted per column.

    ``scale`` < 1 shrinks rows and domain together (rows/domain kept), which keeps
    the per-row join statistics of the full workload.
    """
    rows = max(1, int(10_000_000 * scale))
    domain = max(16, int((1 << 22) * scale))
    return chain(4, rows, domain, 1.1, seed, name="chain4_zipf1.1")


def config3(seed: int = 0x5EED0003, scale: float = 1.0) -> Query:
    """Star: 100M-row fact with 4 FK columns, 4 dims of 1M rows keeping 10%."""
    return star(max(1, int(100_000_000 * scale)), 4, max(10, int(1_000_000 * scale)), 0.1, seed,
                name="star4")


def config4(seed: int = 0x5EED0004, scale: float = 1.0, device: Optional[str] = None) -> Query:
    """Triangle over 50M power-law (gamma 2.1) edges on 2^22 vertices (``device``: see
    powerlaw_edges)."""
    return triangle(max(1, int(50_000_000 * scale)), max(8, int((1 << 22) * scale)), 2.1, seed, device=device)



def config6(seed: int = 0x5EED0006, scale: float = 1.0, k: int = 4) -> Query:
    """The k-clique query (k = 3 or 4) over a directed power-law (gamma 2.5) edge list of
    103,663 edges on 7,066 vertices: the size of the paper's vote network (Section
    3.1.3), which is not available here."""
    src, dst = powerlaw_edges(max(1, int(103_663 * scale)), max(8, int(7_066 * scale)), 2.5, seed)
    q = clique4(src, dst) if k == 4 else clique3(src, dst)
    q.meta.update(nverts=max(8, int(7_066 * scale)), gamma=2.5, seed=seed)
    return q

def tiny_random(seed: int, kind: str = "any") -> Query:
    """Small random instances for brute-force checks: <=5 relations, <=48 rows, tiny domains.

    Covers chains, stars, trees, triangles and 4-cycles, empty relations, single-key
    columns, negative keys and the int32 extremes, self-joins and predicates that keep
    none, some or all rows.
    """
    rng = rng_for(seed, 99, 0, 0)
    kinds = ["chain", "star", "tree", "triangle", "cycle4", "selfjoin", "pair"]
    if kind == "any":
        kind = kinds[int(rng.integers(0, len(kinds)))]
    nrels = {"chain": int(rng.integers(2, 6)), "star": int(rng.integers(3, 6)),
             "tree": int(rng.integers(3, 6)), "triangle": 3, "cycle4": 4,
             "selfjoin": 3, "pair": 2}[kind]
    dom = int(rng.integers(2, 17))
    special = np.array([-2**31, 2**31 - 1, -1, 0, 7], dtype=np.int64)
    mode = int(rng.integers(0, 4))

    def column(n):
        if mode == 0:
            v = rng.integers(0, dom, size=n)
        elif mode == 1:
            v = rng.integers(-dom, dom, size=n)
        elif mode == 2:
            v = special[rng.integers(0, min(len(special), max(2, dom // 3)), size=n)]
        else:
            v = np.full(n, int(rng.integers(-3, 3)))
        return v.astype(np.int32)

    def nrows():
        r = int(rng.integers(0, 49))
        return 0 if rng.random() < 0.06 else r

    rels = []
    if kind == "selfjoin":
        n = nrows()
        a, b = column(n), column(n)
        rels = [Relation(f"E{i}", [a, b]) for i in range(3)]
        edges = [(0, 1, 1, 0), (1, 1, 2, 0)]
        if rng.random() < 0.5:
            edges.append((2, 1, 0, 0))
    else:
        for i in range(nrels):
            n = nrows()
            ncols = int(rng.integers(1, 4))
            rels.append(Relation(f"R{i}", [column(n) for _ in range(ncols)]))
        edges = []
        for i in range(1, nrels):
            if kind in ("chain", "triangle", "cycle4", "pair"):
                p = i - 1
            elif kind == "star":
                p = 0
            else:
                p = int(rng.integers(0, i))
            edges.append((p, int(rng.integers(0, len(rels[p].cols))), i,
                          int(rng.integers(0, len(rels[i].cols)))))
        if kind in ("triangle", "cycle4"):
            edges.append((nrels - 1, int(rng.integers(0, len(rels[-1].cols))), 0,
                          int(rng.integers(0, len(rels[0].cols)))))
        perm = rng.permutation(len(edges))
        edges = [edges[j] for j in perm]
    for r in rels:
        u = rng.random()
        if u < 0.3 and r.nrows >= 0:
            c = int(rng.integers(0, len(r.cols)))
            lo = int(rng.integers(-dom, dom))
            hi = lo + int(rng.integers(0, 2 * dom + 1))
            r.pred = (c, lo, hi)
    return Query(f"tiny_{kind}_{seed}", rels, edges, 0, dict(kind=kind, seed=seed))
