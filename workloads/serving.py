"""The batched / served query mix: many chain and star joins of uneven sizes.

Each query is drawn from its own seeded stream:
  * kind chain or star with probability 1/2 each, 3..5 relations (uniform);
  * rows per relation log-uniform in [min_rows, max_rows];
  * one Zipf exponent s uniform in [0, s_max] for all its key columns;
  * chain: every column Zipf(s) over a domain of 2^22 keys with its own random
    rank->key permutation, R_t.c1 = R_{t+1}.c0;
  * star: the largest drawn relation is the fact table; dimension j has
    (pk, attr), two random permutations of its rows, and the predicate
    attr < 10% of its rows; fact foreign key j is Zipf(s) over dimension j's rows,
    mapped through a random permutation of them.
A query whose exact result count exceeds a cap is redrawn from the next stream of
its seed chain (`redraw`).

Columns are generated either with numpy on the CPU (`query_cpu`, for checks against
the oracle) or with torch on the GPU (`query_gpu`, for large mixes); the two draw
from different random streams but the same distributions. Nothing here computes any
part of the join or the filters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from . import Query, Relation, rng_for, zipf_ranks

DOMAIN = 1 << 22
KEEP = 0.10


@dataclass
class QuerySpec:
    index: int
    draw: int            # 0 for the first draw, k for the k-th redraw
    kind: str            # "chain" or "star"
    rows: List[int]      # per relation; a star's fact table first
    s: float
    seed: int            # seed of this draw's column streams

    @property
    def input_tuples(self) -> int:
        return int(sum(self.rows))

    def edges(self) -> List[Tuple[int, int, int, int]]:
        n = len(self.rows)
        if self.kind == "chain":
            return [(t, 1, t + 1, 0) for t in range(n - 1)]
        return [(0, j, j + 1, 0) for j in range(n - 1)]


def draw_spec(seed: int, index: int, draw: int = 0, min_rows: int = 10_000, max_rows: int = 20_000_000,
              s_max: float = 1.3) -> QuerySpec:
    rng = rng_for(seed, 5, index, draw)
    kind = "chain" if rng.random() < 0.5 else "star"
    n = int(rng.integers(3, 6))
    lo, hi = math.log(min_rows), math.log(max_rows)
    rows = [int(round(math.exp(rng.uniform(lo, hi)))) for _ in range(n)]
    if kind == "star":
        rows.sort(reverse=True)
    s = float(rng.uniform(0.0, s_max))
    qseed = int(rng.integers(0, 2**62))
    return QuerySpec(index, draw, kind, rows, s, qseed)


def serving_specs(seed: int, n: int = 256, **kw) -> List[QuerySpec]:
    return [draw_spec(seed, i, 0, **kw) for i in range(n)]


def redraw(seed: int, spec: QuerySpec, **kw) -> QuerySpec:
    """The next draw of the same query index (used when its count exceeds the cap)."""
    return draw_spec(seed, spec.index, spec.draw + 1, **kw)


# ---------------------------------------------------------------- numpy (CPU)

def query_cpu(spec: QuerySpec) -> Query:
    n = len(spec.rows)
    rels = []
    if spec.kind == "chain":
        for t in range(n):
            cols = []
            for c in range(2):
                rng = rng_for(spec.seed, t, c, 0)
                r = zipf_ranks(rng, spec.rows[t], DOMAIN, spec.s)
                perm = rng_for(spec.seed, t, c, 1).permutation(DOMAIN)
                cols.append(perm[r].astype(np.int32))
            rels.append(Relation("R%d" % t, cols))
    else:
        fcols = []
        for j in range(1, n):
            rng = rng_for(spec.seed, 0, j, 0)
            r = zipf_ranks(rng, spec.rows[0], spec.rows[j], spec.s)
            fcols.append(rng_for(spec.seed, 0, j, 1).permutation(spec.rows[j])[r].astype(np.int32))
        rels.append(Relation("F", fcols))
        for j in range(1, n):
            pk = rng_for(spec.seed, j, 0, 1).permutation(spec.rows[j]).astype(np.int32)
            attr = rng_for(spec.seed, j, 1, 1).permutation(spec.rows[j]).astype(np.int32)
            rels.append(Relation("D%d" % j, [pk, attr], pred=(1, 0, int(round(KEEP * spec.rows[j])))))
    return Query("%s%d_q%d" % (spec.kind, n, spec.index), rels, spec.edges(), 0,
                 dict(kind=spec.kind, s=spec.s, seed=spec.seed))


# ---------------------------------------------------------------- torch (GPU)

def _zipf_gpu(torch, g, n: int, domain: int, s: float, device):
    if s == 0.0:
        return torch.randint(0, domain, (n,), generator=g, device=device)
    w = torch.arange(1, domain + 1, dtype=torch.float64, device=device).pow_(-s)
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    u = torch.rand(n, generator=g, dtype=torch.float64, device=device)
    return torch.searchsorted(cdf, u, right=True).clamp_(max=domain - 1)


def query_gpu(spec: QuerySpec, device="cuda:0"):
    """(relations, edges) with relations as [(list of int32 device tensors, pred)]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(spec.seed)
    n = len(spec.rows)
    rels = []
    if spec.kind == "chain":
        for t in range(n):
            cols = []
            for _ in range(2):
                r = _zipf_gpu(torch, g, spec.rows[t], DOMAIN, spec.s, device)
                perm = torch.randperm(DOMAIN, generator=g, device=device)
                cols.append(perm[r].to(torch.int32).contiguous())
            rels.append((cols, None))
    else:
        fcols = []
        for j in range(1, n):
            r = _zipf_gpu(torch, g, spec.rows[0], spec.rows[j], spec.s, device)
            perm = torch.randperm(spec.rows[j], generator=g, device=device)
            fcols.append(perm[r].to(torch.int32).contiguous())
        rels.append((fcols, None))
        for j in range(1, n):
            pk = torch.randperm(spec.rows[j], generator=g, device=device).to(torch.int32)
            attr = torch.randperm(spec.rows[j], generator=g, device=device).to(torch.int32)
            rels.append(([pk, attr], (1, 0, int(round(KEEP * spec.rows[j])))))
    return rels, spec.edges()
