"""The serving extension: a query's result is the same alone and in a mix.

A mix of small chain and star queries (the batched workload's distributions at
small sizes, generated on the CPU) runs once alone, one plan at a time, and then
through servers whose arena is small enough that admission has to wait: all queries
at once, then staggered while others run. Count, checksum and every tuple must be
identical; counts and checksums also equal the oracle's. Failure handling: a query
whose workspace exceeds the arena is refused at submit, one whose result can never
fit fails alone, and an unsupported cyclic shape fails while its neighbours finish.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from workloads import serving as S
from sjtest import lexsort_rows, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=5)
SEED = 0x5EED0005


@pytest.fixture(scope="module")
def mix():
    specs = S.serving_specs(SEED, n=20, min_rows=500, max_rows=60_000)
    out = []
    ctx = sj.Context(0)
    for sp in specs:
        q = S.query_cpu(sp)
        rels = to_device(q)
        plan = sj.Plan(ctx, rels, q.edges, root=q.root, eager=True, **OPTS)
        plan.build_filters()
        plan.sieve()
        cnt, chk = plan.join()
        tup = plan.result().cpu().numpy().copy()
        _, rcnt, rchk = oracle.hash_join(q)
        assert (cnt, chk) == (rcnt, rchk), sp
        out.append((sp, q, rels, (cnt, chk), tup, plan.workspace_bytes))
    torch.cuda.synchronize()
    return out


def run_server(mix, arena_bytes, slots, stagger):
    """Submit every query (optionally staggered), then collect each result as soon as
    its query finishes and release it at once, as a serving client does."""
    srv = sj.Server(arena_bytes, slots=slots)
    try:
        tickets = []
        for i, (sp, q, rels, _, _, _) in enumerate(mix):
            tickets.append(srv.submit(rels, q.edges, root=q.root, **OPTS))
            if stagger and i % 3 == 2:
                time.sleep(0.002)
        results = {}
        peak = 0
        deadline = time.time() + 120
        while len(results) < len(tickets):
            assert time.time() < deadline, "queries did not finish"
            progressed = False
            for t in tickets:
                if t in results:
                    continue
                info = srv.info(t)
                if info["state"] in (sj.SJ_QUERY_DONE, sj.SJ_QUERY_FAILED):
                    assert info["state"] == sj.SJ_QUERY_DONE, info
                    results[t] = (info, srv.result(t).cpu().numpy().copy())
                    peak = max(peak, srv.stats()["arena_peak"])
                    srv.release(t)
                    progressed = True
            if not progressed:
                time.sleep(0.001)
        assert srv.stats()["arena_used"] == 0
        return [results[t] for t in tickets], peak
    finally:
        srv.close()


@pytest.mark.parametrize("slots,stagger", [(4, False), (3, True), (1, False)])
def test_served_equals_alone(mix, slots, stagger):
    biggest = max(m[5] for m in mix)
    res_bytes = max(m[3][0] * len(m[1].rels) * 4 for m in mix)
    arena = 2 * (biggest + res_bytes) + (1 << 20)   # at most a couple of queries at a time
    results, peak = run_server(mix, arena, slots, stagger)
    assert peak <= arena
    for (sp, q, _, cc, tup, _), (info, got) in zip(mix, results):
        assert (info["count"], info["checksum"]) == cc, sp
        assert got.shape == tup.shape and np.array_equal(got, tup), sp
        assert info["t_submit_ns"] <= info["t_admit_ns"] <= info["t_done_ns"]


@pytest.fixture(scope="module")
def bigq():
    """A chain with a large result (about 2000^3 / 200^2 tuples) and its alone run."""
    bq = W.chain(3, 2000, 200, 0.0, 77)
    brels = to_device(bq)
    bplan = sj.Plan(sj.Context(0), brels, bq.edges, root=bq.root, eager=True, **OPTS)
    bplan.build_filters()
    bplan.sieve()
    bcc = bplan.join()
    torch.cuda.synchronize()
    assert bcc[0] * 3 * 4 > 65536
    return (None, bq, brels, bcc, None, bplan.workspace_bytes)


def test_server_count_only_and_failures(mix, bigq):
    sp, q, rels, cc, _, wsb = mix[0]
    # a workspace larger than the whole arena is refused at submit
    tiny = sj.Server(1 << 16, slots=2)
    try:
        with pytest.raises(sj.SjError) as e:
            tiny.submit(rels, q.edges, root=q.root, **OPTS)
        assert e.value.code == sj.SJ_ERR_NOMEM
    finally:
        tiny.close()
    # a result that can never fit beside its workspace fails alone; count-only and
    # fitting neighbours finish with the right answers; an unsupported cyclic shape
    # fails (or, if it is an executed shape, finishes)
    big = bigq
    arena = big[5] + 4096
    fits = [m for m in mix if m[5] + m[3][0] * len(m[1].rels) * 4 + 512 <= arena]
    counts_only = [m for m in mix if m[5] <= arena]
    assert fits and counts_only
    srv = sj.Server(arena, slots=1)
    try:
        t_big = srv.submit(big[2], big[1].edges, root=big[1].root, **OPTS)
        t_fit = [(m, srv.submit(m[2], m[1].edges, root=m[1].root, **OPTS)) for m in fits[:4]]
        t_cnt = [(m, srv.submit(m[2], m[1].edges, root=m[1].root, count_only=True, **OPTS)) for m in counts_only[:4]]
        cyc = W.tiny_random(31, kind="cycle4")
        t_cyc = srv.submit(to_device(cyc), cyc.edges, root=cyc.root, **OPTS)
        i_big = srv.info(t_big, wait=True)
        assert i_big["state"] == sj.SJ_QUERY_FAILED and i_big["status"] == sj.SJ_ERR_CAPACITY, i_big
        assert (i_big["count"], i_big["checksum"]) == big[3]
        srv.release(t_big)
        for m, t in t_fit:   # each result is consumed and released before the next is awaited
            info = srv.info(t, wait=True)
            assert info["state"] == sj.SJ_QUERY_DONE, info
            assert (info["count"], info["checksum"]) == m[3]
            assert np.array_equal(srv.result(t).cpu().numpy(), m[4])
            srv.release(t)
        for m, t in t_cnt:
            info = srv.info(t, wait=True)
            assert info["state"] == sj.SJ_QUERY_DONE and (info["count"], info["checksum"]) == m[3], info
            srv.release(t)
        i_cyc = srv.info(t_cyc, wait=True)
        if i_cyc["state"] == sj.SJ_QUERY_FAILED:
            assert i_cyc["status"] == sj.SJ_ERR_UNSUPPORTED, i_cyc
        else:
            _, rc, rk = oracle.hash_join(cyc)
            assert (i_cyc["count"], i_cyc["checksum"]) == (rc, rk)
        srv.release(t_cyc)
        assert srv.stats()["arena_used"] == 0
    finally:
        srv.close()


def test_unreleased_results_fail_the_next_query_instead_of_hanging(bigq):
    """A result the client does not release keeps the arena full: the next query gets
    its workspace but no room for its result, and fails with SJ_ERR_NOMEM after the
    bounded wait instead of waiting forever."""
    m = bigq
    arena = m[5] + m[3][0] * len(m[1].rels) * 4 + 4096
    srv = sj.Server(arena, slots=1)
    try:
        t1 = srv.submit(m[2], m[1].edges, root=m[1].root, **OPTS)
        assert srv.info(t1, wait=True)["state"] == sj.SJ_QUERY_DONE   # its result now holds the arena
        t2 = srv.submit(m[2], m[1].edges, root=m[1].root, **OPTS)
        i2 = srv.info(t2, wait=True)
        assert i2["state"] == sj.SJ_QUERY_FAILED and i2["status"] == sj.SJ_ERR_NOMEM, i2
        srv.release(t1)
        srv.release(t2)
    finally:
        srv.close()


def test_full_arena_of_waiting_results_requeues_instead_of_failing(bigq):
    """Two slots whose workspaces fill the arena but leave no room for a second result:
    every running query ends up waiting for result memory, so the one admitted last gives
    its workspace back and runs again later. Every query finishes DONE with the answer it
    has alone (the client releases each result as soon as it is done)."""
    m = bigq
    ws = (m[5] + 255) // 256 * 256
    res = (m[3][0] * len(m[1].rels) * 4 + 255) // 256 * 256
    arena = 2 * ws + res - 256
    srv = sj.Server(arena, slots=2)
    try:
        tickets = [srv.submit(m[2], m[1].edges, root=m[1].root, **OPTS) for _ in range(4)]
        done = {}
        deadline = time.time() + 120
        while len(done) < len(tickets):
            assert time.time() < deadline, "queries did not finish"
            for t in tickets:
                if t in done:
                    continue
                info = srv.info(t)
                if info["state"] in (sj.SJ_QUERY_DONE, sj.SJ_QUERY_FAILED):
                    assert info["state"] == sj.SJ_QUERY_DONE, info
                    assert (info["count"], info["checksum"]) == m[3]
                    done[t] = info
                    srv.release(t)
            time.sleep(0.001)
        assert sum(i["requeues"] for i in done.values()) >= 1
        assert srv.stats()["arena_used"] == 0
    finally:
        srv.close()


@pytest.mark.parametrize("flag", [sj.SJ_FLAG_FAULT_FILTERS, sj.SJ_FLAG_FAULT_SIEVE, sj.SJ_FLAG_FAULT_JOIN,
                                  sj.SJ_FLAG_FAULT_RESULT])
def test_injected_device_error_fails_one_query_only(mix, flag):
    """A query whose phase reports SJ_ERR_DEVICE (injected on the host, no device fault)
    fails alone with that status and message; every other query in the mix finishes with
    the count, checksum and tuples it has alone (which equal the oracle's)."""
    bad = [i for i, m in enumerate(mix) if m[3][0] > 0][1]   # a non-empty result reaches the result phase
    srv = sj.Server(8 << 30, slots=4)
    try:
        tickets = [srv.submit(m[2], m[1].edges, root=m[1].root, flags=flag if i == bad else 0, **OPTS)
                   for i, m in enumerate(mix)]
        for i, (m, t) in enumerate(zip(mix, tickets)):
            info = srv.info(t, wait=True)
            if i == bad:
                assert info["state"] == sj.SJ_QUERY_FAILED and info["status"] == sj.SJ_ERR_DEVICE, info
                assert "injected" in info["error"]
            else:
                assert info["state"] == sj.SJ_QUERY_DONE, info
                assert (info["count"], info["checksum"]) == m[3]
                assert np.array_equal(srv.result(t).cpu().numpy(), m[4])
            srv.release(t)
        assert srv.stats()["arena_used"] == 0
    finally:
        srv.close()


def test_served_value_tuples(mix):
    """Queries served in value mode return the oracle's result projected to values."""
    srv = sj.Server(8 << 30, slots=3)
    try:
        tickets = [srv.submit(m[2], m[1].edges, root=m[1].root, values=True, **OPTS) for m in mix[:8]]
        for m, t in zip(mix[:8], tickets):
            info = srv.info(t, wait=True)
            assert info["state"] == sj.SJ_QUERY_DONE, info
            want = oracle.project(m[1], m[4].astype(np.uint32))
            assert np.array_equal(srv.result(t).cpu().numpy(), want)
            srv.release(t)
    finally:
        srv.close()


def test_stored_mix_sample_served_equals_oracle():
    """The measured serving mix at its stated sizes (rows in [10^4, 2*10^7]): its 24
    smallest queries, served together, return the count and checksum that the oracle
    stored for them (tests/golden/serving_mix.json, written by make_serving_golden.py
    with oracle.join_tree_dp), and every tuple of oracle.hash_join (their results hold
    at most a few thousand tuples)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "serving_mix.json")) as fh:
        doc = json.load(fh)
    ents = sorted(doc["queries"], key=lambda e: sum(e["rows"]))[:24]
    specs = [S.draw_spec(doc["seed"], e["index"], e["draw"], min_rows=doc["min_rows"], max_rows=doc["max_rows"])
             for e in ents]
    for sp, e in zip(specs, ents):
        assert (sp.kind, list(sp.rows)) == (e["kind"], list(e["rows"])), e["index"]
    srv = sj.Server(8 << 30, slots=4)
    try:
        tickets = []
        for sp in specs:
            rel_t, edges = S.query_gpu(sp)
            tickets.append(srv.submit([sj.Rel(c, p) for c, p in rel_t], edges, root=0, **OPTS))
        for sp, e, t in zip(specs, ents, tickets):
            info = srv.info(t, wait=True)
            assert info["state"] == sj.SJ_QUERY_DONE, (e["index"], info)
            assert (info["count"], info["checksum"]) == (e["count"], e["checksum"]), e["index"]
            got = srv.result(t).cpu().numpy().astype(np.int64)
            want, _, _ = oracle.hash_join(S.query_cpu(sp))
            assert np.array_equal(lexsort_rows(got), lexsort_rows(np.asarray(want, dtype=np.int64))), e["index"]
            srv.release(t)
    finally:
        srv.close()
