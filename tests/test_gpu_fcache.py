"""The filter catalogue: backward filters reused across queries (Section 2.3).

A reused filter must hold exactly the bits the plan would have built, so every check
here is the plain parity bar: survivor lists and filter words equal the oracle's,
count, checksum and tuples equal the oracle's join, with and without reuse. On top of
that: which filters are reused (a repeated query reuses all of its backward filters,
a query containing an answered sub-join reuses that sub-join's filters, a change of
options, predicate, root or data does not hit), that reused builds are not launched,
eviction, a catalogue too small for anything, cyclic queries (the tree's filters
reused, the closing filter rebuilt) and a server whose workers share one catalogue.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from workloads import serving as S
from sjtest import check_sieve, check_sorted_in_preorder, lexsort_rows, to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=11)


@pytest.fixture(scope="module")
def chain5():
    q = W.chain(5, [3000, 4000, 5000, 3000, 2000], 2000, 0.5, 0x5EED00F1)
    rels = to_device(q)
    ref = oracle.hash_join(q)
    return q, rels, ref


def run(plan):
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    tup = plan.result().cpu().numpy().astype(np.uint32)
    return cnt, chk, tup


def check(q, plan, ref, opts=OPTS):
    """Count, checksum, tuples (as a set; the order is the plan's preorder), survivors, filters."""
    cnt, chk, tup = run(plan)
    assert (cnt, chk) == (ref[1], ref[2])
    assert np.array_equal(lexsort_rows(tup), lexsort_rows(ref[0]))
    check_sorted_in_preorder(q, tup)
    check_sieve(q, plan, **opts)


def bwd_how(plan):
    """{relation: how its backward filter is held}."""
    out = {}
    for f in range(plan.filter_count()):
        d = plan.filter_desc(f, nblocks=False)
        if d["kind"] == sj.SJ_FILTER_BACKWARD:
            out[d["index"]] = plan.filter_cached(f)
    return out


def test_repeated_query_reuses_every_backward_filter(chain5):
    q, rels, ref = chain5
    cache = sj.FilterCache(8 << 20)
    p1 = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **OPTS)
    assert bwd_how(p1) == {1: 2, 2: 2, 3: 2, 4: 2}
    check(q, p1, ref)
    st = cache.stats()
    assert (st["misses"], st["hits"], st["entries"]) == (4, 0, 4)
    # a second plan on another stream, profiled: reuses all four, launches none of their builds
    s2 = torch.cuda.Stream()
    p2 = sj.Plan(sj.Context(0, stream=s2), rels, q.edges, root=0, filter_cache=cache, profile=True, **OPTS)
    assert bwd_how(p2) == {1: 1, 2: 1, 3: 1, 4: 1}
    with torch.cuda.stream(s2):
        check(q, p2, ref)
    labels = [e["label"] for e in p2.profile()]
    assert not [l for l in labels if l.startswith("bfb_") and ":bwd:" in l], labels
    assert [l for l in labels if l.startswith("bfb_")], "forward filters are still built"
    assert cache.stats()["hits"] == 4
    # the producing plan's later calls (recorded anew without the builds) stay exact
    for _ in range(2):
        check(q, p1, ref)
    del p1, p2
    assert cache.stats()["pinned"] == 0
    cache.close()


def test_sub_join_filters_reused_by_a_larger_query(chain5):
    """Q1 = R3 join R4 join R5 rooted at R3; Q2 = the whole chain rooted at R1 contains it:
    the filters of R4 and R5 (and only those) are reused."""
    q, rels, ref = chain5
    q1 = W.Query("sub", q.rels[2:], [(0, 1, 1, 0), (1, 1, 2, 0)], 0)
    ref1 = oracle.hash_join(q1)
    cache = sj.FilterCache(8 << 20)
    p1 = sj.Plan(sj.Context(0), rels[2:], q1.edges, root=0, filter_cache=cache, **OPTS)
    check(q1, p1, ref1)
    p2 = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **OPTS)
    assert bwd_how(p2) == {1: 2, 2: 2, 3: 1, 4: 1}
    check(q, p2, ref)
    st = cache.stats()
    assert (st["hits"], st["misses"], st["entries"]) == (2, 4, 4)


def test_changed_inputs_do_not_hit(chain5):
    q, rels, ref = chain5
    cache = sj.FilterCache(8 << 20)
    base = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **OPTS)
    check(q, base, ref)
    del base
    # other options
    for change in (dict(bits_per_key=12), dict(k=4), dict(block_bits=256), dict(seed=12), dict(passes=1)):
        opts = dict(OPTS, **change)
        p = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **opts)
        assert set(bwd_how(p).values()) == {2}, change
        check(q, p, ref, opts)
    # a predicate on the leaf changes its filter and every filter above it
    qp = W.Query("pred", [W.Relation(r.name, r.cols, r.pred) for r in q.rels], q.edges, 0)
    qp.rels[4].pred = (1, 0, 1000)
    relsp = list(rels)
    relsp[4] = sj.Rel(rels[4].cols, (1, 0, 1000))
    p = sj.Plan(sj.Context(0), relsp, q.edges, root=0, filter_cache=cache, **OPTS)
    assert set(bwd_how(p).values()) == {2}
    check(qp, p, oracle.hash_join(qp))
    # another root: other build columns
    qr = W.Query("rev", q.rels, q.edges, 4)
    p = sj.Plan(sj.Context(0), rels, q.edges, root=4, filter_cache=cache, **OPTS)
    assert set(bwd_how(p).values()) == {2}
    check(qr, p, oracle.hash_join(qr))
    del p
    # invalidating the leaf's build column drops the leaf's filter and all above it
    p = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **OPTS)
    assert set(bwd_how(p).values()) == {1}
    del p
    cache.invalidate(rels[4].cols[0])
    p = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **OPTS)
    assert set(bwd_how(p).values()) == {2}
    check(q, p, ref)
    del p
    cache.clear()
    assert cache.stats()["entries"] == 0
    p = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **OPTS)
    assert set(bwd_how(p).values()) == {2}
    check(q, p, ref)


def test_eviction_and_a_catalogue_too_small(chain5):
    q, rels, ref = chain5
    # the four backward filters need about 3.5 KiB + 256 B each; room for about three
    cache = sj.FilterCache(3 * 4096)
    seen_evict = False
    for seed in (21, 22, 23):
        opts = dict(OPTS, seed=seed)
        p = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **opts)
        check(q, p, ref, opts)
        assert 0 in bwd_how(p).values()   # what did not fit is built in the workspace
        del p
        st = cache.stats()
        assert st["used_bytes"] <= st["capacity_bytes"]
        seen_evict |= st["evictions"] > 0
    assert seen_evict and cache.stats()["uncached"] > 0
    tiny = sj.FilterCache(512)
    p = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=tiny, **OPTS)
    assert set(bwd_how(p).values()) == {0}
    check(q, p, ref)
    assert tiny.stats()["uncached"] == 4


def test_cyclic_query_reuses_tree_filters_and_rebuilds_the_closing_filter():
    q = W.triangle(20000, 1500, 2.1, 0x5EED00F2)
    rels = to_device(q)
    rc, rk = oracle.triangle_cycles(*q.rels[0].cols)
    cache = sj.FilterCache(8 << 20)
    for it in range(2):
        p = sj.Plan(sj.Context(0), rels, q.edges, root=0, filter_cache=cache, **OPTS)
        hows = {}
        for f in range(p.filter_count()):
            d = p.filter_desc(f, nblocks=False)
            hows.setdefault(d["kind"], set()).add(p.filter_cached(f))
        assert hows[sj.SJ_FILTER_BACKWARD] == {2 if it == 0 else 1}
        assert hows[sj.SJ_FILTER_CLOSING] == {0}
        assert hows[sj.SJ_FILTER_FORWARD] == {0}
        p.build_filters()
        p.sieve()
        check_sieve(q, p, **OPTS)
        assert p.join() == (rc, rk)


def test_attach_states_and_lifetime(chain5):
    q, rels, ref = chain5
    cache = sj.FilterCache(8 << 20)
    p = sj.Plan(sj.Context(0), rels, q.edges, root=0, **OPTS)
    check(q, p, ref)
    p.use_filter_cache(cache)          # back to the bound state: filters must be built again
    with pytest.raises(sj.SjError) as e:
        p.sieve()
    assert e.value.code == sj.SJ_ERR_STATE
    check(q, p, ref)
    with pytest.raises(sj.SjError) as e:   # a plan still holds entries
        cache.close()
    assert e.value.code == sj.SJ_ERR_STATE
    p.use_filter_cache(None)
    assert set(bwd_how(p).values()) == {0}
    check(q, p, ref)
    torch.cuda.synchronize()
    cache.close()


def test_server_workers_share_one_catalogue(chain5):
    """The same queries twice through a server attached to a catalogue: the second
    round reuses every backward filter; a query submitted many times at once is
    answered correctly whether its filters are built, reused or duplicated."""
    specs = S.serving_specs(0x5EED00F3, n=8, min_rows=500, max_rows=20_000)
    mix = [chain5]
    for sp in specs:
        qq = S.query_cpu(sp)
        mix.append((qq, to_device(qq), oracle.hash_join(qq)))
    nbwd = sum(len(qq.rels) - 1 for qq, _, _ in mix)
    cache = sj.FilterCache(64 << 20)
    srv = sj.Server(256 << 20, slots=3)
    srv.use_filter_cache(cache)
    try:
        for rnd in range(2):
            tickets = [srv.submit(r, qq.edges, root=qq.root, **OPTS) for qq, r, _ in mix]
            for (qq, _, ref), t in zip(mix, tickets):
                info = srv.info(t, wait=True)
                assert info["state"] == sj.SJ_QUERY_DONE, info
                assert (info["count"], info["checksum"]) == (ref[1], ref[2])
                assert np.array_equal(srv.result(t).cpu().numpy().astype(np.uint32), ref[0])
                srv.release(t)
            st = cache.stats()
            if rnd == 0:
                assert st["misses"] == nbwd and st["hits"] == 0, st
            else:
                assert st["hits"] == nbwd, st
        qq, r, ref = mix[0]
        cache.clear()
        tickets = [srv.submit(r, qq.edges, root=qq.root, **OPTS) for _ in range(6)]
        for t in tickets:
            info = srv.info(t, wait=True)
            assert info["state"] == sj.SJ_QUERY_DONE and (info["count"], info["checksum"]) == (ref[1], ref[2])
            assert np.array_equal(srv.result(t).cpu().numpy().astype(np.uint32), ref[0])
            srv.release(t)
    finally:
        srv.close()
    assert cache.stats()["pinned"] == 0
    cache.close()


def test_plan_outlives_its_context_and_stream(chain5):
    """A plan attached to the catalogue is destroyed after its context and after the
    caller has destroyed the context's stream (a raw HIP stream): releasing its entries
    must not touch that stream. Another query on the same catalogue then reuses the
    entries and still equals the oracle."""
    import ctypes
    q, rels, ref = chain5
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    cache = sj.FilterCache(64 << 20)
    stream = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(stream)) == 0
    torch.cuda.synchronize()
    ctx = sj.Context(0, stream=torch.cuda.ExternalStream(stream.value))
    plan = sj.Plan(ctx, rels, q.edges, filter_cache=cache, **OPTS)
    check(q, plan, ref)
    assert hip.hipStreamSynchronize(stream) == 0
    sj.lib().sj_ctx_destroy(ctx.handle)      # the caller's context first (the plan keeps it alive) ...
    ctx.handle = None
    assert hip.hipStreamDestroy(stream) == 0  # ... then its stream ...
    del plan                                 # ... then the plan, which lets go of its entries
    again = sj.Plan(sj.Context(0), rels, q.edges, filter_cache=cache, **OPTS)
    assert set(bwd_how(again).values()) == {1}
    check(q, again, ref)
    del again
    cache.close()
