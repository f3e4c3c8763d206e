"""Autotuner for the batched / served query mix: filter parameters and the sieve's
partition of rows over workgroups.

Bits per key, the number of hashes k and the block size trade filter size and probe
cost against false positives, which surviving rows then cost in the join; the number
of workgroups a sieve probe splits its rows over (each takes a contiguous share) trades
parallelism against per-workgroup set-up for small relations. The best choice depends
on the query's shape, size and skew, so it is measured:

    python -m paper_2308_16370_amd.autotune --out paper_2308_16370_amd/tuning.json

draws sample queries from the batched workload's distributions (on the GPU), runs
each with every candidate (bits_per_key, k, block_bits, probe_grid) and times the
whole query the way the server runs it: a new plan, its launches made one by one
(eager), filters, sieve, count pass and materialisation. For each bucket (kind,
decade of total input rows, low or high skew) it keeps the candidate with the least
total time over the bucket's samples. `choose` reads the table; buckets it has not
seen fall back to the nearest size decade of the same kind and skew, then to the
defaults. Every candidate gives the same exact result, so the choice changes only the
time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")
DEFAULT = (8, 6, 512, 256)
CANDIDATES = [(b, k, B, g) for b in (6, 8, 12, 16) for k in (2, 4, 6) for B in (256, 512) for g in (128, 256)
              if k <= b]

_table_cache: Optional[dict] = None


def bucket(kind: str, input_rows: int, s: float) -> str:
    decade = int(math.floor(math.log10(max(10, input_rows))))
    return "%s/%d/%s" % (kind, decade, "hi" if s >= 0.65 else "lo")


def load(path: str = TABLE) -> dict:
    global _table_cache
    if _table_cache is None or path != TABLE:
        t = {}
        if os.path.exists(path):
            with open(path) as fh:
                t = json.load(fh).get("buckets", {})
        if path != TABLE:
            return t
        _table_cache = t
    return _table_cache


def choose(kind: str, input_rows: int, s: float, table: Optional[dict] = None) -> Tuple[int, int, int, int]:
    """(bits_per_key, k, block_bits, probe_grid) for a query."""
    t = load() if table is None else table
    key = bucket(kind, input_rows, s)
    if key not in t:
        kind_, dec, sk = key.split("/")
        near = [(abs(int(k.split("/")[1]) - int(dec)), k) for k in t
                if k.split("/")[0] == kind_ and k.split("/")[2] == sk]
        if not near:
            return DEFAULT
        key = min(near)[1]
    best = list(t[key]["best"])
    return tuple(best + list(DEFAULT[len(best):]))   # tables written before probe_grid: the default


def _time_query(sj, torch, rels, edges, root, opts, reps: int) -> Tuple[float, Tuple[int, int]]:
    """Seconds per query as the server runs it (a new eager plan each time)."""
    ctx = sj.Context(0)

    def once(out=None):
        plan = sj.Plan(ctx, rels, edges, root=root, eager=True, **opts)
        plan.build_filters()
        plan.sieve()
        cc = plan.join()
        if out is None:
            out = torch.empty((max(cc[0], 1), len(rels)), dtype=torch.int32, device="cuda:0")
        plan.result(out)
        del plan
        return cc, out

    cc, out = once()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        once(out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    del out
    return dt, cc


def tune(seed: int, samples: int, min_rows: int, max_rows: int, reps: int, count_cap: int,
         log=print) -> dict:
    import torch

    import paper_2308_16370_amd as sj
    from workloads import serving as S

    per_bucket: Dict[str, List] = {}
    drawn = 0
    i = 0
    while drawn < samples:
        sp = S.draw_spec(seed, 100000 + i, 0, min_rows=min_rows, max_rows=max_rows)
        i += 1
        rel_t, edges = S.query_gpu(sp)
        rels = [sj.Rel(cols, pred) for cols, pred in rel_t]
        times = {}
        ref = None
        skip = False
        for cand in CANDIDATES:
            opts = dict(bits_per_key=cand[0], k=cand[1], block_bits=cand[2], probe_grid=cand[3], passes=2, seed=1)
            try:
                dt, cc = _time_query(sj, torch, rels, edges, 0, opts, reps)
            except sj.SjError:
                skip = True
                break
            if cc[0] > count_cap:
                skip = True
                break
            if ref is None:
                ref = cc
            if cc != ref:
                raise RuntimeError("candidate %r changed the result of query %d" % (cand, sp.index))
            times[cand] = dt
        del rels, rel_t
        torch.cuda.empty_cache()
        if skip:
            continue
        drawn += 1
        key = bucket(sp.kind, sp.input_tuples, sp.s)
        per_bucket.setdefault(key, []).append(times)
        best = min(times, key=times.get)
        log("query %3d %-14s %9d rows s=%.2f best %r %.3f ms (default %.3f ms)" %
            (sp.index, key, sp.input_tuples, sp.s, best, times[best] * 1e3, times[DEFAULT] * 1e3))
    out = {}
    for key, runs in sorted(per_bucket.items()):
        tot = {c: sum(r[c] for r in runs) for c in CANDIDATES}
        best = min(tot, key=tot.get)
        out[key] = {"best": list(best), "samples": len(runs), "total_ms": round(tot[best] * 1e3, 3),
                    "default_total_ms": round(tot[DEFAULT] * 1e3, 3)}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--seed", type=lambda x: int(x, 0), default=0x5EED0A70)
    ap.add_argument("--samples", type=int, default=48)
    ap.add_argument("--min-rows", type=int, default=10_000)
    ap.add_argument("--max-rows", type=int, default=20_000_000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--count-cap", type=int, default=1 << 26)
    args = ap.parse_args(argv)
    buckets = tune(args.seed, args.samples, args.min_rows, args.max_rows, args.reps, args.count_cap,
                   log=lambda s: print(s, flush=True))
    doc = {"about": "best (bits_per_key, k, block_bits, probe_grid) per (kind, decade of input rows, skew) "
                    "bucket, each query timed as the server runs it (new eager plan), measured by "
                    "paper_2308_16370_amd.autotune",
           "candidates": [list(c) for c in CANDIDATES], "seed": args.seed, "samples": args.samples,
           "buckets": buckets}
    with open(args.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(buckets, indent=1))


if __name__ == "__main__":
    sys.exit(main())
