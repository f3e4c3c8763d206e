"""The star, triangle, synthetic (P-syn) and small-chain workloads beside the headline
chain (used by bench.py).

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


def triangle(steps: int = 3, warmup: int = 1, scale: float = 1.0, binary_cycles: bool = False, log=print) -> Dict:
    import torch

    import paper_2308_16370_amd as sj
    import workloads as W

    t = time.perf_counter()
    q = W.config4(scale=scale, device="cuda:0")
    log("# triangle generated in %.1f s" % (time.perf_counter() - t))
    dev = torch.device("cuda:0")
    cols = [torch.from_numpy(c).to(dev) for c in q.rels[0].cols]
    rels = [sj.Rel(cols) for _ in range(3)]
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=0x5EED0004, binary_cycles=binary_cycles)
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
                        "count and checksum, %s" % (q.rels[0].nrows, q.meta["nverts"],
                                                    "binary plan" if binary_cycles else "intersection walk"),
            "input_tuples": q.input_tuples, "ms_per_step": round(dt * 1e3, 3), "tuples_per_s": q.input_tuples / dt,
            "result_tuples": ref[0], "checksum": ref[1], "intersection_walk_ms": round(walk_ms, 3)}


def cliques(steps: int = 10, warmup: int = 2, log=print) -> Dict:
    """The 3-clique and 4-clique queries of the paper's vote-network experiment (Section
    3.1.3) on a power-law stand-in of the network's size (103,663 edges, 7,066 vertices):
    whole query (filters, sieve, intersection count, tuples written), count and checksum
    compared with the oracle's stored values (tests/golden/clique_wiki.json)."""
    import json
    import os

    import torch

    import paper_2308_16370_amd as sj
    import workloads as W

    g = None
    gpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                         "clique_wiki.json")
    if os.path.exists(gpath):
        with open(gpath) as fh:
            g = json.load(fh)
    dev = torch.device("cuda:0")
    ctx = sj.Context(0)
    out = {}
    for k in (3, 4):
        q = W.config6(k=k)
        cols = [torch.from_numpy(c).to(dev) for c in q.rels[0].cols]
        rels = [sj.Rel(cols) for _ in q.rels]
        plan = sj.Plan(ctx, rels, q.edges, bits_per_key=8, k=6, block_bits=512, passes=2, seed=q.meta["seed"])
        plan.build_filters()
        plan.sieve()
        ref = plan.join()
        buf = torch.empty((ref[0], len(q.rels)), dtype=torch.int32, device=dev)
        got = []

        def step():
            plan.build_filters()
            plan.sieve()
            got.append(plan.join())
            plan.result(buf)

        dt = _timed(step, steps, warmup)
        if any(x != ref for x in got):
            raise RuntimeError("clique%d: the count changed between steps" % k)
        key = "clique%d" % k
        check = None
        if g is not None and g["edges"] == q.rels[0].nrows and g["seed"] == q.meta["seed"]:
            want = (g[key]["count"], g[key]["checksum"])
            if ref != want:
                raise RuntimeError("%s: %r, the oracle's stored value %r" % (key, ref, want))
            check = "count and checksum equal the oracle's stored value (tests/golden/clique_wiki.json)"
        out[key] = {"workload": "%d-clique over %d power-law edges (gamma 2.5) on %d vertices, intersection walk, "
                                "tuples written" % (k, q.rels[0].nrows, q.meta["nverts"]),
                    "input_tuples": q.input_tuples, "ms_per_query": round(dt * 1e3, 3),
                    "result_tuples": ref[0], "checksum": ref[1], "check": check}
        del plan, buf
        torch.cuda.empty_cache()
    return out


def psyn(steps: int = 10, warmup: int = 2, M: int = 10_000_000, r: int = 10_000, d: int = 10,
         seed: int = 0x5EED0006, log=print) -> Dict:
    """The paper's synthetic R join S join T (Section 3.1.1) at its comparison sizes:
    M = 10^7, r = 10^4, d = 10 (about 2e8 input rows, r * d^3 = 10^7 result tuples,
    materialised). Count and checksum are compared with the closed form r * d^3 and the
    stored oracle value (tests/golden/psyn_full.json) when it was written for these sizes."""
    import json
    import os

    import torch

    import paper_2308_16370_amd as sj
    import workloads as W

    t = time.perf_counter()
    q = W.psyn(M, r, d, seed=seed)
    log("# psyn generated in %.1f s" % (time.perf_counter() - t))
    dev = torch.device("cuda:0")
    rels = [sj.Rel([torch.from_numpy(c).to(dev) for c in rel.cols], rel.pred) for rel in q.rels]
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=seed)
    plan = sj.Plan(sj.Context(0), rels, q.edges, **opts)
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    out = torch.empty((max(cnt, 1), 3), dtype=torch.int32, device=dev)

    def step():
        plan.build_filters()
        plan.sieve()
        plan.join_async()
        plan.result_async(out)

    dt = _timed(step, steps, warmup)
    if plan.join_wait() != (cnt, chk, sj.SJ_OK):
        raise RuntimeError("psyn: the result changed between steps")
    check = "count %s the closed form r*d^3" % ("equals" if cnt == r * d ** 3 else "DIFFERS FROM")
    gold = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                        "psyn_full.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        if (g["M"], g["r"], g["d"], g["seed"]) == (M, r, d, seed):
            check += "; count and checksum %s the stored oracle value" % (
                "equal" if (g["count"], g["checksum"]) == (cnt, chk) else "DIFFER FROM")
    del plan, out
    torch.cuda.empty_cache()
    return {"workload": "psyn: R(%d) join S(%d) join T(%d) on one attribute, M=%d r=%d d=%d, tuples materialised"
                        % (q.rels[0].nrows, q.rels[1].nrows, q.rels[2].nrows, M, r, d),
            "input_tuples": q.input_tuples, "ms_per_step": round(dt * 1e3, 3), "tuples_per_s": q.input_tuples / dt,
            "result_tuples": cnt, "checksum": chk, "check": check}


def chain3_latency(runs: int = 50, warmup: int = 5, log=print) -> Dict:
    """The small 3-way chain (3 x 100k rows, uniform keys over [0, 50000), 10 bits/key,
    k = 7): launch-bound, so its latency per query is reported (whole query through
    recorded graphs, timed to the host having count, checksum and tuples), with the
    oracle's count and checksum beside it."""
    import torch

    import oracle
    import paper_2308_16370_amd as sj
    import workloads as W

    q = W.config1()
    dev = torch.device("cuda:0")
    rels = [sj.Rel([torch.from_numpy(c).to(dev) for c in rel.cols], rel.pred) for rel in q.rels]
    plan = sj.Plan(sj.Context(0), rels, q.edges, bits_per_key=10, k=7, block_bits=512, passes=2, seed=0x5EED0001)
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    out = torch.empty((cnt + 1, 3), dtype=torch.int32, device=dev)
    lat = []
    for i in range(warmup + runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.build_filters()
        plan.sieve()
        plan.join_async()
        plan.result_async(out)
        got = plan.join_wait()
        if i >= warmup:
            lat.append((time.perf_counter() - t) * 1e3)
        if got != (cnt, chk, sj.SJ_OK):
            raise RuntimeError("chain3: the result changed between runs")
    _, rcnt, rchk = oracle.hash_join(q)
    lat.sort()
    return {"workload": "chain3: 3 x 100000 rows, int32 keys uniform over [0, 50000), 10 bits/key k=7, "
                        "tuples materialised", "input_tuples": q.input_tuples, "result_tuples": cnt,
            "latency_ms_p50": round(lat[len(lat) // 2], 4), "latency_ms_min": round(lat[0], 4),
            "latency_ms_p99": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4),
            "check": "count and checksum equal the oracle" if (rcnt, rchk) == (cnt, chk) else "MISMATCH"}


def _whole_query_ms(plan, out, steps: int, warmup: int) -> float:
    def step():
        plan.build_filters()
        plan.sieve()
        plan.join_async()
        plan.result_async(out)
    return _timed(step, steps, warmup) * 1e3


def planner_check(q, opts: Dict, steps: int = 10, warmup: int = 2, log=print) -> Dict:
    """The planner (Section 2.1, Eq. (1)-(3)) on workload q before it runs: estimated
    survivors beside the measured ones for `opts`, and the options it chooses, timed
    beside `opts` (the result is the same with either)."""
    import torch

    import paper_2308_16370_amd as sj
    from . import planner

    t = time.perf_counter()
    st = planner.column_stats(q)
    t_stats = time.perf_counter() - t
    est = planner.estimate(st, q.edges, q.root, opts["bits_per_key"], opts["k"], opts["block_bits"], opts["passes"])
    best = planner.choose(st, q.edges, q.root)
    dev = torch.device("cuda:0")
    rels = [sj.Rel([torch.from_numpy(c).to(dev) for c in r.cols], r.pred) for r in q.rels]
    res = {}
    for name, o in (("given", opts), ("chosen", dict(opts, bits_per_key=best.bits_per_key, k=best.k,
                                                      passes=best.passes))):
        plan = sj.Plan(sj.Context(0), rels, q.edges, root=q.root, **o)
        plan.build_filters()
        surv = plan.sieve(survivors=True)
        cc = plan.join()
        out = torch.empty((max(cc[0], 1), len(q.rels)), dtype=torch.int32, device=dev)
        ms = _whole_query_ms(plan, out, steps, warmup)
        if plan.join_wait() != (cc[0], cc[1], sj.SJ_OK):
            raise RuntimeError("planner check: the result changed between steps")
        res[name] = {"options": {k: o[k] for k in ("bits_per_key", "k", "block_bits", "passes")},
                     "ms_per_step": round(ms, 4), "count": cc[0], "checksum": cc[1], "survivors": surv}
        del plan, out
    if (res["given"]["count"], res["given"]["checksum"]) != (res["chosen"]["count"], res["chosen"]["checksum"]):
        raise RuntimeError("planner check: the chosen options changed the result")
    res["estimated_survivors_given"] = [round(x) for x in est.survivors]
    res["estimate_over_measured"] = [round(e / max(1, m), 3) for e, m in zip(est.survivors, res["given"]["survivors"])]
    res["stats_seconds"] = round(t_stats, 2)
    log("# planner: chose bpk %d k %d passes %d: %.3f ms vs %.3f ms given" % (
        best.bits_per_key, best.k, best.passes, res["chosen"]["ms_per_step"], res["given"]["ms_per_step"]))
    torch.cuda.empty_cache()
    return res


def bloomjoin(steps: int = 10, warmup: int = 2, log=print) -> Dict:
    """n = 2, the Bloomjoin of Section 2.1: the first two relations of the 4-way chain
    (10M rows each, Zipf(1.1) keys over 2^22), a filter on R2's join column sieves R1
    (one pass, the paper's default), then the join and the materialisation. Also the
    Eq. (1) estimate of R1's survivors beside the measured number."""
    import torch

    import paper_2308_16370_amd as sj
    import workloads as W
    from . import planner

    full = W.config2()
    q = W.Query("bloomjoin_n2", full.rels[:2], [full.edges[0]], 0, full.meta)
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=1, seed=0x5EED0002)
    dev = torch.device("cuda:0")
    rels = [sj.Rel([torch.from_numpy(c).to(dev) for c in r.cols], r.pred) for r in q.rels]
    plan = sj.Plan(sj.Context(0), rels, q.edges, **opts)
    plan.build_filters()
    surv = plan.sieve(survivors=True)
    cnt, chk = plan.join()
    out = torch.empty((max(cnt, 1), 2), dtype=torch.int32, device=dev)
    ms = _whole_query_ms(plan, out, steps, warmup)
    if plan.join_wait() != (cnt, chk, sj.SJ_OK):
        raise RuntimeError("bloomjoin: the result changed between steps")
    st = planner.column_stats(q)
    est = planner.estimate(st, q.edges, 0, 8, 6, 512, 1)
    del plan, out
    torch.cuda.empty_cache()
    return {"workload": "bloomjoin n=2: R1(10M) join R2(10M), Zipf(1.1) over 2^22, 8 bits/key k=6, one pass, "
                        "tuples materialised", "input_tuples": q.input_tuples, "ms_per_step": round(ms, 4),
            "tuples_per_s": q.input_tuples / (ms / 1e3), "result_tuples": cnt, "checksum": chk,
            "survivors": surv, "estimated_survivors": [round(x) for x in est.survivors]}


def main(argv=None) -> int:
    """python -m paper_2308_16370_amd.configbench star|triangle|psyn|chain3|bloomjoin|cliques [--steps K]
    [--scale F] [--binary-cycles]: one workload, one JSON line."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="time one of the side workloads")
    ap.add_argument("workload", choices=["star", "triangle", "psyn", "chain3", "bloomjoin", "cliques"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--scale", type=float, default=1.0, help="triangle: edges and vertices scaled together")
    ap.add_argument("--binary-cycles", action="store_true", help="triangle: count with the binary plan")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    kw = {} if args.steps is None else {"steps": args.steps}
    if args.workload == "triangle":
        kw.update(scale=args.scale, binary_cycles=args.binary_cycles)
    if args.workload == "chain3":
        kw = {} if args.steps is None else {"runs": args.steps}
    fn = {"star": star, "triangle": triangle, "psyn": psyn, "chain3": chain3_latency,
          "bloomjoin": bloomjoin, "cliques": cliques}[args.workload]
    res = fn(log=log, **kw)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
