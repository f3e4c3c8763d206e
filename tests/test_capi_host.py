"""Host-side checks of the C ABI (no GPU needed): exported symbols, plan validation
and the call-order state machine. sj_plan is host-only, so fake (aligned, non-null)
device addresses exercise it without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sievejoin.h")
LIB = os.path.join(ROOT, "paper_2308_16370_amd", "libsievejoin.so")

if not os.path.exists(LIB):
    pytest.skip("libsievejoin.so not built", allow_module_level=True)

import paper_2308_16370_amd as sj  # noqa: E402


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:sj_status|const char \*)\s*(sj_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(sj.EXPORTED) == names


FAKE = 0x7F0000000000


def mkrels(specs):
    """specs: list of (nrows, ncols, pred) -> (_Rel array, keepalive)."""
    arr = (sj._Rel * len(specs))()
    keep = []
    addr = FAKE
    for i, (n, nc, pred) in enumerate(specs):
        ptrs = (ctypes.c_void_p * nc)(*[addr + 4096 * j for j in range(nc)])
        addr += 1 << 30
        keep.append(ptrs)
        arr[i].nrows, arr[i].ncols = n, nc
        arr[i].cols = ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p))
        arr[i].pred_col, arr[i].pred_lo, arr[i].pred_hi = pred if pred else (-1, 0, 0)
    return arr, keep


def plan(specs, edges, **kw):
    L = sj.lib()
    ctx = ctypes.c_void_p()
    assert L.sj_ctx_create(0, None, ctypes.byref(ctx)) == 0
    arr, keep = mkrels(specs)
    earr = (sj._Edge * max(1, len(edges)))(*[sj._Edge(*e) for e in edges])
    o = sj._Opts(kw.get("bpk", 0), kw.get("k", 0), kw.get("B", 0), kw.get("passes", 0), 0, kw.get("root", -1),
                 kw.get("flags", 0), kw.get("probe_grid", 0), kw.get("probe_lds", 0))
    p = ctypes.c_void_p()
    ws = ctypes.c_uint64()
    st = L.sj_plan(ctx, arr, len(specs), earr, len(edges), ctypes.byref(o), ctypes.byref(p), ctypes.byref(ws))
    err = L.sj_last_error(ctx).decode()
    return st, p, ws.value, ctx, err


def test_valid_chain_plans():
    st, p, ws, ctx, err = plan([(1000, 2, None)] * 4, [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 3, 0)])
    assert st == 0, err
    assert ws > 4 * 1000 * 4
    nf = ctypes.c_int32()
    assert sj.lib().sj_filter_count(p, ctypes.byref(nf)) == 0
    assert nf.value == 6          # 3 backward + 3 forward
    st, p1, ws1, _, err = plan([(1000, 2, None)] * 4, [(0, 1, 1, 0), (1, 1, 2, 0), (2, 1, 3, 0)], passes=1)
    assert st == 0
    assert sj.lib().sj_filter_count(p1, ctypes.byref(nf)) == 0 and nf.value == 3


@pytest.mark.parametrize("specs,edges,kw,code", [
    ([(10, 2, None)] * 2, [(0, 1, 0, 0)], {}, sj.SJ_ERR_GRAPH),                  # self-edge
    ([(10, 2, None)] * 3, [(0, 1, 1, 0)], {}, sj.SJ_ERR_GRAPH),                  # disconnected
    ([(10, 2, None)] * 2, [(0, 2, 1, 0)], {}, sj.SJ_ERR_GRAPH),                  # bad column
    ([(10, 2, None)] * 2, [(0, 1, 5, 0)], {}, sj.SJ_ERR_GRAPH),                  # bad relation
    ([(10, 2, (3, 0, 1))] * 2, [(0, 1, 1, 0)], {}, sj.SJ_ERR_GRAPH),             # bad predicate column
    ([(10, 2, None)] * 2, [(0, 1, 1, 0)], {"k": 13}, sj.SJ_ERR_INVALID),
    ([(10, 2, None)] * 2, [(0, 1, 1, 0)], {"B": 384}, sj.SJ_ERR_INVALID),
    ([(10, 2, None)] * 2, [(0, 1, 1, 0)], {"passes": 3}, sj.SJ_ERR_INVALID),
    ([(10, 2, None)] * 2, [(0, 1, 1, 0)], {"root": 2}, sj.SJ_ERR_INVALID),
    ([(10, 2, None)] * 2, [(0, 1, 1, 0)], {"flags": 256}, sj.SJ_ERR_INVALID),
    ([(2**31, 2, None)] * 2, [(0, 1, 1, 0)], {}, sj.SJ_ERR_INVALID),
    # nine children on one column: the root's step would probe nine filters
    ([(10, 1, None)] * 10, [(0, 0, i, 0) for i in range(1, 10)], {}, sj.SJ_ERR_UNSUPPORTED),
    # a relation joining on nine columns
    ([(10, 9, None)] + [(10, 1, None)] * 9, [(0, i - 1, i, 0) for i in range(1, 10)], {}, sj.SJ_ERR_UNSUPPORTED),
])
def test_invalid_plans(specs, edges, kw, code):
    st, p, ws, ctx, err = plan(specs, edges, **kw)
    assert st == code, err
    assert err


def test_eight_children_accepted():
    st, p, ws, ctx, err = plan([(10, 1, None)] * 9, [(0, 0, i, 0) for i in range(1, 9)])
    assert st == 0, err
    st, p, ws, ctx, err = plan([(10, 8, None)] + [(10, 1, None)] * 8, [(0, i - 1, i, 0) for i in range(1, 9)])
    assert st == 0, err


def test_plans_outlive_their_context():
    """A context destroyed before its plans stays valid for them (a garbage collector may
    release the two in either order)."""
    L = sj.lib()
    st, p, ws, ctx, err = plan([(1000, 2, None)] * 3, [(0, 1, 1, 0), (1, 1, 2, 0)])
    assert st == 0, err
    st2, p2, _, _, _ = plan([(10, 2, None)] * 2, [(0, 1, 1, 0)])
    assert L.sj_ctx_destroy(ctx) == 0
    nf = ctypes.c_int32()
    assert L.sj_filter_count(p, ctypes.byref(nf)) == 0 and nf.value == 4
    assert L.sj_plan_destroy(p) == 0
    assert L.sj_plan_destroy(p2) == 0


def test_misaligned_column_rejected():
    L = sj.lib()
    ctx = ctypes.c_void_p()
    L.sj_ctx_create(0, None, ctypes.byref(ctx))
    arr, keep = mkrels([(10, 1, None), (10, 1, None)])
    bad = (ctypes.c_void_p * 1)(FAKE + 4)
    arr[1].cols = ctypes.cast(bad, ctypes.POINTER(ctypes.c_void_p))
    earr = (sj._Edge * 1)(sj._Edge(0, 0, 1, 0))
    p, ws = ctypes.c_void_p(), ctypes.c_uint64()
    assert L.sj_plan(ctx, arr, 2, earr, 1, None, ctypes.byref(p), ctypes.byref(ws)) == sj.SJ_ERR_INVALID


def test_state_machine_and_workspace_size():
    st, p, ws, ctx, err = plan([(100, 2, None)] * 3, [(0, 1, 1, 0), (1, 1, 2, 0)])
    L = sj.lib()
    assert st == 0
    assert L.sj_build_filters(p) == sj.SJ_ERR_STATE
    assert L.sj_sieve(p, None) == sj.SJ_ERR_STATE
    assert L.sj_join(p, None, None) == sj.SJ_ERR_STATE
    assert L.sj_result(p, None, 0, sj.SJ_RIDS) == sj.SJ_ERR_STATE
    assert L.sj_bind_workspace(p, ctypes.c_void_p(FAKE), ws - 1) == sj.SJ_ERR_NOMEM
    assert L.sj_bind_workspace(p, ctypes.c_void_p(FAKE + 64), ws) == sj.SJ_ERR_INVALID
    assert L.sj_bind_workspace(p, ctypes.c_void_p(FAKE), ws) == 0
    assert L.sj_join(p, None, None) == sj.SJ_ERR_STATE
    assert L.sj_plan_destroy(p) == 0


def test_projection_and_footprint():
    """sj_plan_set_projection checks every (relation, column) pair and the width limit;
    sj_plan_footprint reports the workspace at once and the result size only once the
    count is known."""
    st, p, ws, ctx, err = plan([(100, 2, None), (50, 3, None), (70, 1, None)], [(0, 1, 1, 0), (1, 2, 2, 0)])
    assert st == 0
    L = sj.lib()
    w, wsb, rb = ctypes.c_int32(), ctypes.c_uint64(), ctypes.c_uint64()
    assert L.sj_plan_footprint(p, sj.SJ_RIDS, ctypes.byref(wsb), None, ctypes.byref(w)) == 0
    assert (w.value, wsb.value) == (3, ws)
    assert L.sj_plan_footprint(p, sj.SJ_VALUES, None, None, ctypes.byref(w)) == 0
    assert w.value == 6                                   # every column of every relation
    assert L.sj_plan_footprint(p, sj.SJ_RIDS, None, ctypes.byref(rb), None) == sj.SJ_ERR_STATE
    assert L.sj_plan_footprint(p, 7, None, None, ctypes.byref(w)) == sj.SJ_ERR_INVALID
    pairs = (ctypes.c_int32 * 6)(0, 0, 1, 2, 2, 0)
    assert L.sj_plan_set_projection(p, pairs, 3) == 0
    assert L.sj_plan_footprint(p, sj.SJ_VALUES, None, None, ctypes.byref(w)) == 0 and w.value == 3
    bad = (ctypes.c_int32 * 2)(1, 3)                       # relation 1 has three columns
    assert L.sj_plan_set_projection(p, bad, 1) == sj.SJ_ERR_GRAPH
    bad = (ctypes.c_int32 * 2)(3, 0)
    assert L.sj_plan_set_projection(p, bad, 1) == sj.SJ_ERR_GRAPH
    assert L.sj_plan_set_projection(p, pairs, sj.SJ_MAX_PROJ + 1) == sj.SJ_ERR_INVALID
    assert L.sj_plan_set_projection(p, None, 0) == 0
    assert L.sj_plan_footprint(p, sj.SJ_VALUES, None, None, ctypes.byref(w)) == 0 and w.value == 6
    assert L.sj_plan_destroy(p) == 0


def test_fault_flags_are_accepted_and_unknown_flags_refused():
    for flag in (sj.SJ_FLAG_FAULT_FILTERS, sj.SJ_FLAG_FAULT_SIEVE, sj.SJ_FLAG_FAULT_JOIN, sj.SJ_FLAG_FAULT_RESULT,
                 sj.SJ_FLAG_SIEVE_TWO_LAUNCHES):
        st, p, ws, ctx, err = plan([(10, 1, None)] * 2, [(0, 0, 1, 0)], flags=flag)
        assert st == 0, err
        sj.lib().sj_plan_destroy(p)
    st, p, ws, ctx, err = plan([(10, 1, None)] * 2, [(0, 0, 1, 0)], flags=256)
    assert st == sj.SJ_ERR_INVALID


def test_probe_launch_shape_options():
    """probe_grid: a power of two in 64..1024 (0: the default); probe_lds: 0, 1 or 2."""
    for g in (0, 64, 128, 256, 512, 1024):
        for lds in (0, 1, 2):
            st, p, ws, ctx, err = plan([(1000, 2, None)] * 3, [(0, 1, 1, 0), (1, 1, 2, 0)], probe_grid=g,
                                       probe_lds=lds)
            assert st == 0, (g, lds, err)
            sj.lib().sj_plan_destroy(p)
    for g in (32, 96, 2048):
        st, p, ws, ctx, err = plan([(10, 1, None)] * 2, [(0, 0, 1, 0)], probe_grid=g)
        assert st == sj.SJ_ERR_INVALID and "probe_grid" in err
    st, p, ws, ctx, err = plan([(10, 1, None)] * 2, [(0, 0, 1, 0)], probe_lds=3)
    assert st == sj.SJ_ERR_INVALID and "probe_lds" in err
