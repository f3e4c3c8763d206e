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
the oracle) or with the large steps on the GPU (`query_gpu`, for large mixes). Both
take the same numpy draws (uniforms, integers, permutations) and the same float64 Zipf
CDF, so their columns are identical; `query_gpu` only moves the inverse-CDF searches and
the permutation gathers to the device. Nothing here computes any part of the join or
the filters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from . import Query, Relation, _zipf_cdf, rng_for, zipf_ranks

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

def _ranks_dev(torch, rng, n: int, domain: int, s: float, device):
    """zipf_ranks(rng, n, domain, s) with the search on `device`: the same draws and CDF."""
    if s == 0.0:
        return torch.from_numpy(rng.integers(0, domain, size=n, dtype=np.int64)).to(device)
    cdf = torch.from_numpy(_zipf_cdf(domain, s)).to(device)
    u = torch.from_numpy(rng.random(n)).to(device)
    r = torch.searchsorted(cdf, u, right=True)
    del u, cdf
    return r.clamp_(max=domain - 1)


def query_gpu(spec: QuerySpec, device="cuda:0"):
    """(relations, edges) with relations as [(list of int32 device tensors, pred)]; the
    columns equal query_cpu(spec)'s."""
    import torch
    n = len(spec.rows)
    rels = []
    if spec.kind == "chain":
        for t in range(n):
            cols = []
            for c in range(2):
                r = _ranks_dev(torch, rng_for(spec.seed, t, c, 0), spec.rows[t], DOMAIN, spec.s, device)
                perm = torch.from_numpy(rng_for(spec.seed, t, c, 1).permutation(DOMAIN)).to(device)
                cols.append(perm[r].to(torch.int32).contiguous())
                del r, perm
            rels.append((cols, None))
    else:
        fcols = []
        for j in range(1, n):
            r = _ranks_dev(torch, rng_for(spec.seed, 0, j, 0), spec.rows[0], spec.rows[j], spec.s, device)
            perm = torch.from_numpy(rng_for(spec.seed, 0, j, 1).permutation(spec.rows[j])).to(device)
            fcols.append(perm[r].to(torch.int32).contiguous())
            del r, perm
        rels.append((fcols, None))
        for j in range(1, n):
            pk = torch.from_numpy(rng_for(spec.seed, j, 0, 1).permutation(spec.rows[j]).astype(np.int32)).to(device)
            attr = torch.from_numpy(rng_for(spec.seed, j, 1, 1).permutation(spec.rows[j]).astype(np.int32)).to(device)
            rels.append(([pk, attr], (1, 0, int(round(KEEP * spec.rows[j])))))
    return rels, spec.edges()
