"""The star and triangle workloads beside the headline chain (used by bench.py).

star      -- fact table of 100M rows with 4 foreign keys, 4 dimensions of 1M rows
             keeping 10% by a range predicate; a step is the whole query
             (filters, sieve, asynchronous count and materialisation) replayed as
             graphs, like the chain's. The dominant kernel's event-timed bandwidth
             comes from a profiled plan on the same workspace.
triangle  -- E join E join E over 50M power-law edges (gamma 2.1, 2^22 vertices),
             closing edge E3.dst = E1.src; a step is filters, sieve and the exact
             count and checksum (the result, about 1.8e9 tuples, is not
             materialised), with the 3-cycle counted by intersection. The binary
             plan's count is not timed at this size (its wedge expansion is about
             1.1e12 probes); the 1/16-size workload times both.

Both report input tuples per second (the sum of the relation instances' rows over
the step time) and the count and checksum of the last step, which must equal the
first step's.
"""
from __future__ import annotations

import time
from typing import Dict


def _timed(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / steps


def star(steps: int = 10, warmup: int = 2, log=print) -> Dict:
    import torch

    import paper_2308_16370_amd as sj
    import workloads as W

    t = time.perf_counter()
    q = W.config3(scale=1.0)
    log("# star generated in %.1f s" % (time.perf_counter() - t))
    dev = torch.device("cuda:0")
    rels = [sj.Rel([torch.from_numpy(c).to(dev) for c in r.cols], r.pred) for r in q.rels]
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=0x5EED0003)
    ctx = sj.Context(0)
    plan = sj.Plan(ctx, rels, q.edges, **opts)
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    out = torch.empty((max(cnt, 1), len(q.rels)), dtype=torch.int32, device=dev)

    def step():
        plan.build_filters()
        plan.sieve()
        plan.join_async()
        plan.result_async(out)

    dt = _timed(step, steps, warmup)
    if plan.join_wait() != (cnt, chk, sj.SJ_OK):
        raise RuntimeError("star: the result changed between steps")
    pplan = sj.Plan(ctx, rels, q.edges, workspace=plan.workspace, profile=True, **opts)
    for i in range(3):
        pplan.build_filters()
        pplan.sieve()
        pplan.join()
        pplan.result(out)
        if i == 0:
            pplan.profile(reset=True)
    prof = [e for e in pplan.profile() if e["alg_bytes"] > 0]
    dom = max(prof, key=lambda e: e["total_ms"] / max(1, e["launches"]))
    avg_s = dom["total_ms"] / dom["launches"] / 1e3
    del pplan, plan
    torch.cuda.empty_cache()
    return {"workload": "star: fact 100M x 4 FK, 4 dims x 1M rows keeping 10%, 8 bits/key k=6, 2 passes",
            "input_tuples": q.input_tuples, "ms_per_step": round(dt * 1e3, 4),
            "tuples_per_s": q.input_tuples / dt, "result_tuples": cnt, "checksum": chk,
            "dominant_kernel": {"label": dom["label"], "avg_us": round(avg_s * 1e6, 2),
                                "alg_bytes": dom["alg_bytes"],
                                "achieved_gbs": round(dom["alg_bytes"] / avg_s / 1e9, 1)}}


def triangle(steps: int = 3, warmup: int = 1, scale: float = 1.0, log=print) -> Dict:
    import torch

    import paper_2308_16370_amd as sj
    import workloads as W

    t = time.perf_counter()
    q = W.config4(scale=scale, device="cuda:0")
    log("# triangle generated in %.1f s" % (time.perf_counter() - t))
    dev = torch.device("cuda:0")
    cols = [torch.from_numpy(c).to(dev) for c in q.rels[0].cols]
    rels = [sj.Rel(cols) for _ in range(3)]
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=0x5EED0004)
    ctx = sj.Context(0)
    plan = sj.Plan(ctx, rels, q.edges, **opts)
    plan.build_filters()
    plan.sieve()
    ref = plan.join()
    got = []

    def step():
        plan.build_filters()
        plan.sieve()
        got.append(plan.join())

    dt = _timed(step, steps, warmup)
    if any(g != ref for g in got):
        raise RuntimeError("triangle: the count changed between steps")
    pplan = sj.Plan(ctx, rels, q.edges, workspace=plan.workspace, profile=True, **opts)
    pplan.build_filters()
    pplan.sieve()
    pplan.join()
    walk_ms = sum(e["total_ms"] for e in pplan.profile() if e["label"] == "tri_count")
    del pplan, plan
    torch.cuda.empty_cache()
    return {"workload": "triangle: E join E join E, %d power-law edges (gamma 2.1) over %d vertices, "
                        "count and checksum" % (q.rels[0].nrows, q.meta["nverts"]),
            "input_tuples": q.input_tuples, "ms_per_step": round(dt * 1e3, 3), "tuples_per_s": q.input_tuples / dt,
            "result_tuples": ref[0], "checksum": ref[1], "intersection_walk_ms": round(walk_ms, 3)}


def main(argv=None) -> int:
    """python -m paper_2308_16370_amd.configbench star|triangle [--steps K]: one workload, one JSON line."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="time the star or the triangle workload")
    ap.add_argument("workload", choices=["star", "triangle"])
    ap.add_argument("--steps", type=int, default=None)
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    fn = star if args.workload == "star" else triangle
    res = fn(log=log) if args.steps is None else fn(steps=args.steps, log=log)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
