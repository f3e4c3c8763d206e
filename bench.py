#!/usr/bin/env python3
"""Benchmark of the SieveJoin hot path on one MI355X.

Workload: 4-way chain R1(a,b) join R2(b,c) join R3(c,d) join R4(d,e), 10M rows per
table, int32 keys Zipf(s=1.1) over 2^22 values with an independent random
rank->key permutation per (table, column); blocked Bloom filters of 8 bits per
key, k = 6, 512-bit blocks; backward and forward pruning passes; exact result
count, checksum and materialised int32 row-id tuples.

One step = sj_build_filters + sj_sieve + sj_join_async + sj_result_async on a plan
whose inputs and workspace are already resident in HBM: the exact count stays on the
device and the materialisation reads it there, so the steps queue back to back; the
count, checksum and result status are checked after the warm-up steps and after the
timed ones. The metric is input tuples per
second (the sum of the four relations' rows divided by the step time).

Printed: one JSON line with the contract's fields plus
  roofline      -- for the kernel launch with the longest average duration among those
                   with an algorithmic-byte model: its bytes per launch over its
                   HIP-event-timed average duration, against 8 TB/s HBM; traffic is the
                   HBM bytes per launch from the committed rocprofv3 counter summary
                   (profiles/traffic.json) when it was taken on the current sources;
  launch_groups -- the modelled groups of several launches (each relation's bucketing:
                   radix passes, gather and directory; each DP's two launches), longest
                   first, with their bytes over their event-timed durations;
  cpu_baseline  -- the CPU oracle (plain single-threaded binary hash join) on the
                   same input, timed on this host.

The per-launch event timings come from a second plan on the same workspace that
launches eagerly with an event pair around each kernel (the timed plan replays
recorded graphs); the kernels and data are the same.

configs       -- the small 3-way chain's latency, the star (100M-row fact table), the
                 full-size triangle (50M edges, 3-cycles counted by intersection), the
                 paper's synthetic join at its sizes (2e8 rows, 10^7 tuples), the n=2
                 Bloomjoin, the planner's estimates, and the 3-clique and 4-clique
                 queries on a vote-network-sized graph, timed the same way
                 (paper_2308_16370_amd/configbench.py).
sieve_roofline -- every probe, compaction and filter-build launch of a step: their
                 algorithmic bytes over their summed event-timed durations, against the
                 60% target.
filter_reuse  -- the same step on a plan attached to a filter catalogue, whose
                 backward filters are built once and then reused (their builds drop
                 out of the step); reported beside the headline value, which always
                 builds every filter.

--copy-mib N appends one plain device-to-device copy of N MiB (after the JSON line
is printed) so that a counter run can calibrate FETCH_SIZE / WRITE_SIZE.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# launch groups of the profiling plan that hold several kernels
MULTI_LAUNCH = ("buckets", "dp", "pairs", "tri_count", "k4_count", "clique_write", "cyclic_count", "cyclic_write")


def lib_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2308_16370_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(label):
    """HBM bytes per launch of the launch `label` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("source_hash") != lib_source_hash():
        return None
    for e in t.get("entries", [t]):
        if e.get("label") == label:
            return e.get("bytes_per_launch")
    return None


def host_cpu():
    """The measuring host's CPU model and logical CPU count."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def copy_bandwidth(dev, mib: int = 1024, reps: int = 10):
    """Device-to-device copy of `mib` MiB, timed with torch events on its stream: bytes
    read plus bytes written per second (GB/s)."""
    import torch
    x = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / reps
    del x, y
    return 2.0 * (mib << 20) / sec / 1e9


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=lambda x: int(x, 0), default=0x5EED0002)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink rows and key domain together (tests)")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0, help="append a plain copy of this many MiB")
    ap.add_argument("--no-serve", action="store_true", help="skip the batched / served query mix")
    ap.add_argument("--no-configs", action="store_true", help="skip the star and triangle workloads")
    ap.add_argument("--passes", type=int, default=2, help="sieve passes: 1 (the paper's backward pass) or 2")
    ap.add_argument("--probe-grid", type=int, default=0, help="workgroups per sieve probe launch (0: library default)")
    ap.add_argument("--probe-lds", type=int, default=0, help="LDS filter reservation mode of the probes (0, 1, 2)")
    ap.add_argument("--sieve-two-launches", action="store_true",
                    help="each sieve step as a probe and a compaction launch (SJ_FLAG_SIEVE_TWO_LAUNCHES)")
    ap.add_argument("--serve-queries", type=int, default=256)
    ap.add_argument("--serve-max-rows", type=int, default=20_000_000)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-arena-gb", type=int, default=24)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (asked for %d GPUs)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2308_16370_amd as sj
    import workloads as W

    t_gen = time.perf_counter()
    q = W.config2(seed=args.seed, scale=args.scale)
    t_gen = time.perf_counter() - t_gen
    print("# generated %s: %d relations x %d rows in %.1fs" % (q.name, len(q.rels), q.rels[0].nrows, t_gen),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    rels = [sj.Rel([torch.from_numpy(c).to(dev) for c in r.cols], r.pred) for r in q.rels]
    opts = dict(bits_per_key=8, k=6, block_bits=512, passes=args.passes, seed=args.seed, probe_grid=args.probe_grid,
                probe_lds=args.probe_lds, flags=sj.SJ_FLAG_SIEVE_TWO_LAUNCHES if args.sieve_two_launches else 0)
    ctx = sj.Context(0)
    plan = sj.Plan(ctx, rels, q.edges, **opts)

    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    out = torch.empty((max(cnt, 1), len(q.rels)), dtype=torch.int32, device=dev)
    plan.result(out)
    torch.cuda.synchronize()

    def step():
        # the count stays on the device: the materialisation reads it there, so a step is
        # four recorded graphs replayed back to back with no host round trip
        plan.build_filters()
        plan.sieve()
        plan.join_async()
        plan.result_async(out)

    def check():
        c = plan.join_wait()
        if c != (cnt, chk, sj.SJ_OK):
            raise RuntimeError("result changed between steps: %r vs %r" % (c, (cnt, chk)))

    for _ in range(args.warmup):
        step()
        check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    check()   # the last step's count, checksum and result status
    ms = (t1 - t0) / args.steps * 1e3
    value = q.input_tuples / (ms / 1e3)
    print("# %d steps, %.3f ms/step, count %d" % (args.steps, ms, cnt), file=sys.stderr, flush=True)

    # phase times with torch events (the plan launches on torch's current stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    phases = {"build_filters": 0.0, "sieve": 0.0, "join": 0.0, "result": 0.0}
    for _ in range(args.profile_steps):
        ev[0].record()
        plan.build_filters()
        ev[1].record()
        plan.sieve()
        ev[2].record()
        plan.join()
        ev[3].record()
        plan.result(out)
        ev[4].record()
        torch.cuda.synchronize()
        for i, k in enumerate(phases):
            phases[k] += ev[i].elapsed_time(ev[i + 1]) / args.profile_steps

    # per-kernel HIP-event timings on the same stream, same workspace
    pplan = sj.Plan(ctx, rels, q.edges, workspace=plan.workspace, profile=True, **opts)
    for i in range(args.profile_steps + 1):
        pplan.build_filters()
        pplan.sieve()
        pplan.join()
        pplan.result(out)
        if i == 0:
            pplan.profile(reset=True)
    prof = pplan.profile()
    del pplan
    kernels = sorted(prof, key=lambda e: -e["total_ms"] / max(1, e["launches"]))
    for e in kernels:
        print("# launch group %-28s %8.2f us  %12d algorithmic bytes"
              % (e["label"], e["total_ms"] / max(1, e["launches"]) * 1e3, e["alg_bytes"]), file=sys.stderr)
    # the roofline is for one kernel (one launch per group, so that the rocprofv3 trace
    # shows the same duration); groups of several launches (a relation's bucketing: the
    # radix passes, gather and directory; a DP's two launches) are reported beside it
    modelled = [e for e in kernels if e["alg_bytes"] > 0 and e["label"].split(":")[0] not in MULTI_LAUNCH]
    dom = modelled[0] if modelled else None
    groups = []
    for e in kernels:
        if e["alg_bytes"] > 0 and e["label"].split(":")[0] in MULTI_LAUNCH:
            avg_s = e["total_ms"] / max(1, e["launches"]) / 1e3
            gbs = e["alg_bytes"] / avg_s / 1e9
            groups.append({"label": e["label"], "avg_us": round(avg_s * 1e6, 2), "alg_bytes": e["alg_bytes"],
                           "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
    copy_gbs = copy_bandwidth(dev)
    roofline = None
    if dom:
        avg_s = dom["total_ms"] / dom["launches"] / 1e3
        achieved = dom["alg_bytes"] / avg_s / 1e9
        traffic = load_traffic(dom["label"])
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom["label"],
                    "alg_bytes_per_launch": dom["alg_bytes"], "avg_us": round(avg_s * 1e6, 2),
                    "copy_kernel_gbs": round(copy_gbs, 1)}
    # the result: the materialisation's output launch (the expansion of the root), with
    # the launches before it (the tables of the factorised materialisation, and the
    # decode that writes only when a table does not fit its scratch)
    result_roofline = None
    res = next((e for e in prof if e["label"] == "materialize" and e["alg_bytes"] > 0), None)
    if res:
        avg_s = res["total_ms"] / res["launches"] / 1e3
        ach = res["alg_bytes"] / avg_s / 1e9
        result_roofline = {"bound": "hbm", "kernel": "materialize", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": res["alg_bytes"],
                           "avg_us": round(avg_s * 1e6, 2), "traffic": load_traffic("materialize"),
                           "other_launches_us": {e["label"]: round(e["total_ms"] / max(1, e["launches"]) * 1e3, 2)
                                                 for e in prof if e["label"].startswith("mat_")}}
    # the sieve passes together (every probe, compaction and filter-build launch of a
    # step): their algorithmic bytes over their summed event-timed durations
    sieve = [e for e in prof if e["label"].split(":")[0] in ("probe", "compact", "bfb_hist", "bfb_scan",
                                                              "bfb_scatter", "bfb_region", "count_pred")]
    sieve_ms = sum(e["total_ms"] for e in sieve) / max(1, args.profile_steps)
    sieve_bytes = sum(e["alg_bytes"] for e in sieve)
    sieve_roofline = {"bound": "hbm", "achieved": round(sieve_bytes / (sieve_ms / 1e3) / 1e9, 1) if sieve_ms else None,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "launches_per_step": len(sieve),
                      "alg_bytes_per_step": sieve_bytes, "ms_per_step": round(sieve_ms, 4), "target_frac": 0.6}
    if sieve_ms:
        sieve_roofline["frac"] = round(sieve_roofline["achieved"] / HBM_PEAK_GBS, 4)

    # the same step with the backward filters held in a filter catalogue (built on the
    # first call, reused after): not the headline value, which builds every filter
    cache = sj.FilterCache(256 << 20)
    rplan = sj.Plan(ctx, rels, q.edges, workspace=plan.workspace, filter_cache=cache, **opts)
    rplan.build_filters()
    rplan.sieve()
    if rplan.join() != (cnt, chk):
        raise RuntimeError("the plan attached to the filter catalogue changed the result")
    reused = sum(1 for f in range(rplan.filter_count()) if rplan.filter_cached(f) != 0)
    for _ in range(args.warmup):
        rplan.build_filters()
        rplan.sieve()
        rplan.join_async()
        rplan.result_async(out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rplan.build_filters()
        rplan.sieve()
        rplan.join_async()
        rplan.result_async(out)
    torch.cuda.synchronize()
    ms_reuse = (time.perf_counter() - t0) / args.steps * 1e3
    if rplan.join_wait() != (cnt, chk, sj.SJ_OK):
        raise RuntimeError("the plan attached to the filter catalogue changed the result")
    filter_reuse = {"ms_per_step": round(ms_reuse, 4), "speedup": round(ms / ms_reuse, 3),
                    "filters_in_catalogue": reused, "catalogue_bytes": cache.stats()["used_bytes"]}
    print("# filter catalogue: %.3f ms/step with %d backward filters reused" % (ms_reuse, reused),
          file=sys.stderr, flush=True)
    del rplan

    cpu = None
    check = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        _, rcnt, rchk = oracle.hash_join(q)
        t = time.perf_counter() - t
        cpu = {"value": q.input_tuples / t, "unit": "tuples/s", "cores": 1, "kind": "oracle",
               "sample": "the full workload (4 x %d rows), single-threaded binary hash join, %.2f s"
                         % (q.rels[0].nrows, t),
               "host": host_cpu()}
        check = "count and checksum equal the oracle" if (rcnt, rchk) == (cnt, chk) else "MISMATCH"
        if check == "MISMATCH":
            print("# oracle mismatch: gpu %r oracle %r" % ((cnt, chk), (rcnt, rchk)), file=sys.stderr)

    configs = None
    if not args.no_configs:
        from paper_2308_16370_amd import configbench
        logf = lambda m: print(m, file=sys.stderr, flush=True)
        configs = {"chain3": configbench.chain3_latency(log=logf), "star": configbench.star(log=logf),
                   "triangle": configbench.triangle(log=logf), "psyn": configbench.psyn(log=logf),
                   "bloomjoin_n2": configbench.bloomjoin(log=logf), "cliques": configbench.cliques(log=logf),
                   "planner_chain4": configbench.planner_check(q, opts, log=logf)}
        tri = configs["triangle"]
        gold = os.path.join(ROOT, "tests", "golden", "triangle_cycles.json")
        tri["check"] = "no stored oracle value at this size"
        if os.path.exists(gold):
            with open(gold) as fh:
                cases = [c for c in json.load(fh)["cases"] if abs(c["scale"] - 1.0) < 1e-12]
            if cases:
                ok = (cases[0]["count"], cases[0]["checksum"]) == (tri["result_tuples"], tri["checksum"])
                tri["check"] = "count and checksum equal the stored oracle value" if ok else "MISMATCH"
        logf("# star %.3f ms/step, triangle %.1f ms/step (%s)" % (configs["star"]["ms_per_step"],
                                                                  tri["ms_per_step"], tri["check"]))

    serving = None
    if not args.no_serve:
        from paper_2308_16370_amd import servebench
        del plan
        torch.cuda.empty_cache()
        serving = servebench.run(n=args.serve_queries, max_rows=args.serve_max_rows, slots=args.serve_slots,
                                 arena_bytes=args.serve_arena_gb << 30,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))

    res = {
        "metric": "input tuples/s through sieve+join (4-way chain)",
        "value": value,
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "chain4: 4 x %d rows, int32 keys Zipf(1.1) over %d, per-column permutation, "
                               "blocked Bloom 8 bits/key k=6 512-bit blocks, %d pass%s, tuples materialised"
                               % (q.rels[0].nrows, q.meta["domain"], args.passes, "" if args.passes == 1 else "es"),
                   "input_tuples": q.input_tuples, "result_tuples": cnt, "seed": args.seed,
                   "probe_grid": args.probe_grid or 256, "probe_lds": args.probe_lds,
                   "sieve_launches_per_step": 2 if args.sieve_two_launches else 1},
        "roofline": roofline,
        "sieve_roofline": sieve_roofline,
        "result_roofline": result_roofline,
        "launch_groups": groups[:8],
        "cpu_baseline": cpu,
        "check": check,
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "filter_reuse": filter_reuse,
        "configs": configs,
        "serving": serving,
        "kernels": [{"label": e["label"], "avg_us": round(e["total_ms"] / max(1, e["launches"]) * 1e3, 2),
                     "alg_bytes": e["alg_bytes"]} for e in kernels[:12]],
    }
    print(json.dumps(res), flush=True)
    if args.copy_mib:
        x = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
