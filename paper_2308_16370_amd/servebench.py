"""Batched and served throughput and latency on the query mix (used by bench.py).

The mix (workloads.serving) is generated on the GPU and stays resident. One untimed
pass of the whole mix warms up kernel loading and the workers first. Each query is
first run alone with a count pass; a query whose count exceeds `count_cap` is
redrawn. Filter options come from the autotuner's table per query. Then the same
queries go through sj_server runs over one arena:
  * alone         -- one slot, each query submitted when the previous one has
                     finished: its latency is its own service time;
  * one_at_a_time -- one slot, every query submitted at once: the queries run one
                     after the other, each with the whole GPU (latency includes queueing);
  * burst         -- `slots` slots, every query submitted at once;
  * poisson_<f>   -- `slots` slots, Poisson arrivals at f times the one-at-a-time
                     service rate;
  (batched(): batches recorded into one graph with sj_batch; not run while
   sj_batch_submit is switched off in the library.)
A collector consumes each result as its query finishes (checks count and checksum
against the alone run, which equals the oracle's stored value for the mix when
tests/golden/serving_mix.json holds it, then releases it). Latency is completion minus submission on
the server's clock; throughput counts input tuples over the span from the first
submission to the last completion.
"""
from __future__ import annotations

import threading
import time
from typing import Dict, List, Optional

import numpy as np


def _pct(v: List[float], p: float) -> float:
    return float(np.percentile(np.asarray(v), p)) if v else float("nan")


def load_store(seed: int, n: int, min_rows: int, max_rows: int, count_cap: int, path: Optional[str] = None):
    """The stored oracle values of the mix ({index: entry}) if they were written for
    exactly these parameters (tests/golden/serving_mix.json), else None."""
    import json
    import os
    path = path or os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                                "serving_mix.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        doc = json.load(fh)
    if (doc["seed"], doc["min_rows"], doc["max_rows"], doc["count_cap"]) != (seed, min_rows, max_rows, count_cap):
        return None
    if doc["n"] < n:
        return None
    return {q["index"]: q for q in doc["queries"]}


def prepare(seed: int, n: int, min_rows: int, max_rows: int, count_cap: int, tuned: bool, log=print):
    """Queries of the mix on the GPU, each run alone once. With the stored oracle values
    of the mix, each query takes the stored draw, and its count and checksum alone must
    equal the stored ones (`oracle` in each entry: the stored pair, else None)."""
    import torch

    import paper_2308_16370_amd as sj
    from workloads import serving as S

    from . import autotune

    ctx = sj.Context(0)
    queries = []
    redraws = 0
    store = load_store(seed, n, min_rows, max_rows, count_cap)
    for sp in S.serving_specs(seed, n=n, min_rows=min_rows, max_rows=max_rows):
        if store is not None:
            while sp.draw < store[sp.index]["draw"]:
                sp = S.redraw(seed, sp, min_rows=min_rows, max_rows=max_rows)
                redraws += 1
        while True:
            rel_t, edges = S.query_gpu(sp)
            rels = [sj.Rel(cols, pred) for cols, pred in rel_t]
            b, k, B, g = autotune.choose(sp.kind, sp.input_tuples, sp.s) if tuned else autotune.DEFAULT
            opts = dict(bits_per_key=b, k=k, block_bits=B, probe_grid=g, passes=2, seed=sp.seed & 0xFFFF)
            plan = sj.Plan(ctx, rels, edges, root=0, eager=True, **opts)
            plan.build_filters()
            plan.sieve()
            cc = plan.join()
            del plan
            if cc[0] <= count_cap:
                break
            redraws += 1
            del rels, rel_t
            sp = S.redraw(seed, sp, min_rows=min_rows, max_rows=max_rows)
        ref = None
        if store is not None:
            ent = store[sp.index]
            ref = (ent["count"], ent["checksum"])
            if cc != ref:
                raise RuntimeError("query %d alone: %r, the oracle's stored value %r" % (sp.index, cc, ref))
        queries.append(dict(spec=sp, rels=rels, edges=edges, opts=opts, cc=cc, oracle=ref))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("# mix: %d queries, %d input tuples, %d redraws, %s" % (
        len(queries), sum(q["spec"].input_tuples for q in queries), redraws,
        "every count and checksum alone equals the stored oracle value" if store is not None
        else "no stored oracle values for this mix"))
    return queries, redraws, store is not None


def serve(queries, arena, slots: int, rate: Optional[float], seed: int = 1, sequential: bool = False) -> Dict:
    """Run the mix through a server; rate None: all at once, else Poisson arrivals;
    sequential: each query is submitted when the previous one has finished (its
    latency is then its own service time, with no queueing)."""
    import paper_2308_16370_amd as sj

    srv = sj.Server(0, slots=slots, arena=arena)
    tickets: List[Optional[int]] = [None] * len(queries)
    submitted = threading.Event()
    errors = []

    def submitter():
        try:
            t0 = time.perf_counter()
            gaps = np.random.default_rng(seed).exponential(1.0 / rate, len(queries)) if rate else None
            at = 0.0
            for i, q in enumerate(queries):
                if sequential and i > 0:
                    srv.info(tickets[i - 1], wait=True)
                if rate:
                    at += gaps[i]
                    d = t0 + at - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                tickets[i] = srv.submit(q["rels"], q["edges"], root=0, **q["opts"])
        except Exception as e:   # reported by the collector
            errors.append(e)
        finally:
            submitted.set()

    th = threading.Thread(target=submitter)
    th.start()
    lat, admit, done = [], [], 0
    t_first, t_last = None, None
    mismatches = 0
    pending = set(range(len(queries)))
    while pending:
        if errors:
            raise errors[0]
        progressed = False
        for i in list(pending):
            t = tickets[i]
            if t is None:
                continue
            info = srv.info(t)
            if info["state"] in (sj.SJ_QUERY_DONE, sj.SJ_QUERY_FAILED):
                if info["state"] != sj.SJ_QUERY_DONE:
                    raise RuntimeError("query %d failed: %s" % (i, info["error"]))
                if (info["count"], info["checksum"]) != queries[i]["cc"]:
                    mismatches += 1
                if queries[i]["oracle"] is not None and (info["count"], info["checksum"]) != queries[i]["oracle"]:
                    mismatches += 1
                srv.release(t)
                lat.append((info["t_done_ns"] - info["t_submit_ns"]) / 1e6)
                admit.append((info["t_admit_ns"] - info["t_submit_ns"]) / 1e6)
                t_first = info["t_submit_ns"] if t_first is None else min(t_first, info["t_submit_ns"])
                t_last = info["t_done_ns"] if t_last is None else max(t_last, info["t_done_ns"])
                pending.discard(i)
                progressed = True
        if not progressed:
            time.sleep(0.0002)
    th.join()
    stats = srv.stats()
    srv.close()
    span_s = (t_last - t_first) / 1e9
    tuples = sum(q["spec"].input_tuples for q in queries)
    return {"slots": slots, "queries": len(queries), "span_s": round(span_s, 4),
            "queries_per_s": round(len(queries) / span_s, 2), "tuples_per_s": tuples / span_s,
            "p50_ms": round(_pct(lat, 50), 3), "p99_ms": round(_pct(lat, 99), 3),
            "mean_admit_wait_ms": round(float(np.mean(admit)), 3), "arena_peak_bytes": stats["arena_peak"],
            "equal_results": mismatches == 0}


def batched(queries, batch: int = 16, reps: int = 3, log=print) -> Dict:
    """The mix in batches of `batch` queries, each batch recorded once into one graph
    (sj_batch: every query's filters, sieve, count and materialisation side by side) and
    then replayed `reps` times; the mix's time is the sum of the batches' mean replay
    times. Every query's count and checksum is checked after each replay (against its
    alone run and the stored oracle value)."""
    import torch

    import paper_2308_16370_amd as sj

    total_ms = 0.0
    batch_ms = []
    mismatches = 0
    for b0 in range(0, len(queries), batch):
        group = queries[b0:b0 + batch]
        ctx = sj.Context(0)
        plans = [sj.Plan(ctx, q["rels"], q["edges"], root=0, **q["opts"]) for q in group]
        outs = [torch.empty((max(1, q["cc"][0]), len(q["rels"])), dtype=torch.int32, device="cuda:0") for q in group]
        bt = sj.Batch(ctx, plans)
        bt.submit(outs)                      # records the graph
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            bt.submit(outs)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / reps * 1e3
        for q, p in zip(group, plans):
            got = p.join_wait()
            if got[:2] != q["cc"] or got[2] != sj.SJ_OK or (q["oracle"] is not None and got[:2] != q["oracle"]):
                mismatches += 1
        batch_ms.append(ms)
        total_ms += ms
        del bt, plans, outs
        torch.cuda.empty_cache()
    tuples = sum(q["spec"].input_tuples for q in queries)
    out = {"batch": batch, "batches": len(batch_ms), "span_s": round(total_ms / 1e3, 4),
           "tuples_per_s": tuples / (total_ms / 1e3), "queries_per_s": round(len(queries) / (total_ms / 1e3), 2),
           "batch_ms_p50": round(_pct(batch_ms, 50), 3), "batch_ms_p99": round(_pct(batch_ms, 99), 3),
           "equal_results": mismatches == 0}
    log("# batched (%d per graph): %.3f s for the mix, %.3g tuples/s" % (batch, out["span_s"], out["tuples_per_s"]))
    return out


def run(seed: int = 0x5EED0005, n: int = 256, min_rows: int = 10_000, max_rows: int = 20_000_000,
        slots: int = 8, arena_bytes: int = 24 << 30, lam=(0.5, 0.9, 1.2), count_cap: int = 1 << 26,
        tuned: bool = True, log=print) -> Dict:
    import torch

    queries, redraws, pinned = prepare(seed, n, min_rows, max_rows, count_cap, tuned, log)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    serve(queries, arena, slots, None)   # warm-up: first launches of every kernel, worker start-up
    alone = serve(queries, arena, 1, None, sequential=True)
    log("# alone (each submitted after the previous finished): p50 %.2f ms p99 %.2f ms" % (alone["p50_ms"],
                                                                                          alone["p99_ms"]))
    one = serve(queries, arena, 1, None)
    log("# one at a time: %.3f s, p50 %.2f ms" % (one["span_s"], one["p50_ms"]))
    burst = serve(queries, arena, slots, None)
    log("# burst, %d slots: %.3f s, p50 %.2f ms p99 %.2f ms" % (slots, burst["span_s"], burst["p50_ms"],
                                                                burst["p99_ms"]))
    rate = one["queries_per_s"]
    out = {"queries": len(queries), "input_tuples": sum(q["spec"].input_tuples for q in queries),
           "rows_per_relation": [min_rows, max_rows], "redraws": redraws, "count_cap": count_cap,
           "oracle_check": ("every query's count and checksum, alone and in each served run, equals the stored "
                            "oracle value (tests/golden/serving_mix.json)") if pinned else
                           "no stored oracle values for this mix (results compared with each query alone)",
           "arena_bytes": arena_bytes, "autotuned": tuned, "alone": alone, "one_at_a_time": one, "burst": burst,

           "burst_speedup": round(burst["tuples_per_s"] / one["tuples_per_s"], 3)}
    for f in lam:
        r = serve(queries, arena, slots, f * rate, seed=int(f * 1000))
        r["arrival_rate_qps"] = round(f * rate, 2)
        out["poisson_%g" % f] = r
        log("# poisson %.1fx: p50 %.2f ms p99 %.2f ms" % (f, r["p50_ms"], r["p99_ms"]))
    del arena
    return out
