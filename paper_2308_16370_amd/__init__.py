"""Python binding of the SieveJoin C ABI (include/sievejoin.h) for MI355X.

Argument marshalling only: every step of the sieve and the join runs in the HIP
kernels of ``libsievejoin.so``. PyTorch supplies device memory (input columns, the
plan's workspace, result buffers) and the HIP stream.

    import torch, paper_2308_16370_amd as sj
    ctx = sj.Context()
    plan = sj.Plan(ctx, [sj.Rel([a, b]), sj.Rel([b2, c], pred=(1, 0, 10))],
                   [(0, 1, 1, 0)], bits_per_key=8, k=6)
    plan.build_filters(); plan.sieve()
    count, checksum = plan.join()
    tuples = plan.result()        # int32 [count, nrels] row ids on the GPU

The library must be built first (``__graft_entry__.build()`` or
``python paper_2308_16370_amd/_build.py``); loading fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsievejoin.so")

SJ_OK = 0
SJ_ERR_INVALID = -1
SJ_ERR_GRAPH = -2
SJ_ERR_NOMEM = -3
SJ_ERR_CAPACITY = -4
SJ_ERR_STATE = -5
SJ_ERR_DEVICE = -6
SJ_ERR_UNSUPPORTED = -7
_NAMES = {0: "SJ_OK", -1: "SJ_ERR_INVALID", -2: "SJ_ERR_GRAPH", -3: "SJ_ERR_NOMEM", -4: "SJ_ERR_CAPACITY",
          -5: "SJ_ERR_STATE", -6: "SJ_ERR_DEVICE", -7: "SJ_ERR_UNSUPPORTED"}

SJ_FILTER_BACKWARD = 0
SJ_FILTER_FORWARD = 1
SJ_FILTER_CLOSING = 2

EXPORTED = ["sj_ctx_create", "sj_ctx_set_stream", "sj_ctx_destroy", "sj_last_error", "sj_plan",
            "sj_bind_workspace", "sj_build_filters", "sj_sieve", "sj_join", "sj_result", "sj_join_async",
            "sj_result_async", "sj_join_wait", "sj_plan_destroy",
            "sj_filter_count", "sj_filter_desc", "sj_filter_copy", "sj_survivors_copy", "sj_profile_collect",
            "sj_profile_count", "sj_profile_entry", "sj_profile_reset", "sj_server_create", "sj_server_submit",
            "sj_server_query", "sj_server_release", "sj_server_stats", "sj_server_last_error",
            "sj_server_destroy", "sj_fcache_create", "sj_plan_use_filter_cache", "sj_plan_filter_cached",
            "sj_fcache_invalidate", "sj_fcache_clear", "sj_fcache_stats", "sj_fcache_destroy",
            "sj_server_use_filter_cache", "sj_filter_probe", "sj_filter_insert", "sj_plan_set_projection",
            "sj_plan_footprint", "sj_bind_static_workspace", "sj_batch_create", "sj_batch_submit",
            "sj_batch_destroy", "sj_filter_propagate_scratch", "sj_filter_propagate", "sj_plan_cfilter",
            "sj_cfilter_update", "sj_cfilter_probe", "sj_cfilter_export", "sj_cfilter_apply", "sj_cfilter_destroy"]
SJ_FLAG_PROFILE = 1
SJ_FLAG_EAGER = 2
SJ_FLAG_BINARY_CYCLES = 4
SJ_FLAG_FAULT_FILTERS, SJ_FLAG_FAULT_SIEVE, SJ_FLAG_FAULT_JOIN, SJ_FLAG_FAULT_RESULT = 8, 16, 32, 64
SJ_FLAG_SIEVE_TWO_LAUNCHES = 128
SJ_RIDS, SJ_VALUES = 0, 1
SJ_MAX_PROJ = 32
SJ_STATIC_WORKSPACE_BYTES = 64 << 20
SJ_MAX_SLOTS = 16
SJ_QUERY_QUEUED, SJ_QUERY_RUNNING, SJ_QUERY_DONE, SJ_QUERY_FAILED = 0, 1, 2, 3
SJ_RESULT_TUPLES, SJ_RESULT_COUNT, SJ_RESULT_VALUES = 0, 1, 2


class SjError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class _Rel(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int32),
                ("cols", ctypes.POINTER(ctypes.c_void_p)), ("pred_col", ctypes.c_int32),
                ("pred_lo", ctypes.c_int32), ("pred_hi", ctypes.c_int32)]


class _Edge(ctypes.Structure):
    _fields_ = [("rel_a", ctypes.c_int32), ("col_a", ctypes.c_int32), ("rel_b", ctypes.c_int32),
                ("col_b", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("bits_per_key", ctypes.c_uint32), ("k", ctypes.c_uint32), ("block_bits", ctypes.c_uint32),
                ("passes", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("root", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("probe_grid", ctypes.c_uint32), ("probe_lds", ctypes.c_uint32)]


class _QueryInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("count", ctypes.c_uint64),
                ("checksum", ctypes.c_uint64), ("result_offset", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64), ("slot", ctypes.c_int32),
                ("requeues", ctypes.c_int32), ("error", ctypes.c_char * 160)]


class _FcInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("capacity_bytes", "used_bytes", "entries", "pinned", "hits",
                                              "misses", "uncached", "evictions")]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsievejoin.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, V = ctypes.POINTER, ctypes.c_void_p
        i32, u32, u64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        sig = {
            "sj_ctx_create": [i32, V, P(V)],
            "sj_ctx_set_stream": [V, V],
            "sj_ctx_destroy": [V],
            "sj_plan": [V, P(_Rel), i32, P(_Edge), i32, P(_Opts), P(V), P(u64)],
            "sj_bind_workspace": [V, V, u64],
            "sj_build_filters": [V],
            "sj_sieve": [V, P(u64)],
            "sj_join": [V, P(u64), P(u64)],
            "sj_result": [V, V, u64, i32],
            "sj_join_async": [V],
            "sj_result_async": [V, V, u64, i32],
            "sj_join_wait": [V, P(u64), P(u64), P(i32)],
            "sj_plan_destroy": [V],
            "sj_filter_count": [V, P(i32)],
            "sj_filter_desc": [V, i32, P(i32), P(i32), P(i32), P(i32), P(u32)],
            "sj_filter_copy": [V, i32, V, u64],
            "sj_survivors_copy": [V, i32, V, u64, P(u64)],
            "sj_profile_collect": [V],
            "sj_profile_count": [V, P(i32)],
            "sj_profile_entry": [V, i32, P(ctypes.c_char_p), P(ctypes.c_double), P(u64), P(u64)],
            "sj_profile_reset": [V],
            "sj_server_create": [i32, V, u64, i32, P(V)],
            "sj_server_submit": [V, P(_Rel), i32, P(_Edge), i32, P(_Opts), i32, P(u64)],
            "sj_server_query": [V, u64, i32, P(_QueryInfo)],
            "sj_server_release": [V, u64],
            "sj_server_stats": [V, P(u64), P(u64), P(i32), P(i32)],
            "sj_server_destroy": [V],
            "sj_fcache_create": [i32, V, u64, P(V)],
            "sj_plan_use_filter_cache": [V, V],
            "sj_plan_filter_cached": [V, i32, P(i32)],
            "sj_fcache_invalidate": [V, V],
            "sj_fcache_clear": [V],
            "sj_fcache_stats": [V, P(_FcInfo)],
            "sj_fcache_destroy": [V],
            "sj_server_use_filter_cache": [V, V],
            "sj_filter_probe": [V, i32, V, u64, V, P(u64)],
            "sj_filter_insert": [V, i32, V, u64, V, P(u64)],
            "sj_plan_set_projection": [V, V, i32],
            "sj_plan_footprint": [V, i32, P(u64), P(u64), P(i32)],
            "sj_bind_static_workspace": [V],
            "sj_batch_create": [V, V, i32, P(V)],
            "sj_batch_submit": [V, V, V, i32],
            "sj_batch_destroy": [V],
            "sj_filter_propagate_scratch": [V, i32, u64, P(u64)],
            "sj_filter_propagate": [V, i32, V, u64, V, u64, P(u64)],
            "sj_plan_cfilter": [V, i32, V, u64, P(V)],
            "sj_cfilter_update": [V, V, u64, i32],
            "sj_cfilter_probe": [V, V, u64, V, P(u64)],
            "sj_cfilter_export": [V, V, u64],
            "sj_cfilter_apply": [V, V, i32],
            "sj_cfilter_destroy": [V],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = i32
        L.sj_last_error.argtypes = [V]
        L.sj_last_error.restype = ctypes.c_char_p
        L.sj_server_last_error.argtypes = [V]
        L.sj_server_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Context:
    """sj_ctx on a device, enqueuing on a torch stream (default: the current stream)."""

    def __init__(self, device: int = 0, stream=None):
        self.device = device
        self.handle = ctypes.c_void_p()
        with torch.cuda.device(device):
            s = _stream_handle(stream)
        self._check(lib().sj_ctx_create(device, ctypes.c_void_p(s), ctypes.byref(self.handle)))

    def set_stream(self, stream) -> None:
        self._check(lib().sj_ctx_set_stream(self.handle, ctypes.c_void_p(_stream_handle(stream))))

    def last_error(self) -> str:
        return (lib().sj_last_error(self.handle) or b"").decode()

    def _check(self, code: int) -> None:
        if code != SJ_OK:
            raise SjError(code, self.last_error() if self.handle else "")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.sj_ctx_destroy(h)
            self.handle = None


class Rel:
    """A relation: int32 device column tensors (equal length) and an optional
    predicate ``(col, lo, hi)`` keeping rows with lo <= cols[col][row] < hi."""

    def __init__(self, cols: Sequence[torch.Tensor], pred: Optional[Tuple[int, int, int]] = None):
        self.cols = list(cols)
        self.pred = pred


def _marshal(rels: Sequence[Rel], edges: Sequence[Tuple[int, int, int, int]]):
    """ctypes arrays of sj_rel and sj_edge, plus the pointer arrays they reference."""
    arr = (_Rel * max(1, len(rels)))()
    keep = []
    for i, r in enumerate(rels):
        for c in r.cols:
            if c.dtype != torch.int32 or c.dim() != 1:
                raise ValueError("columns must be 1-D int32 tensors")
        ptrs = (ctypes.c_void_p * len(r.cols))(*[c.data_ptr() if c.numel() else None for c in r.cols])
        keep.append(ptrs)
        arr[i].nrows = r.cols[0].numel() if r.cols else 0
        arr[i].ncols = len(r.cols)
        arr[i].cols = ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p))
        if r.pred is None:
            arr[i].pred_col, arr[i].pred_lo, arr[i].pred_hi = -1, 0, 0
        else:
            arr[i].pred_col, arr[i].pred_lo, arr[i].pred_hi = (int(x) for x in r.pred)
    earr = (_Edge * max(1, len(edges)))(*[_Edge(*[int(x) for x in e]) for e in edges])
    return arr, earr, keep


class Plan:
    """sj_plan plus its workspace (a torch uint8 tensor on the context's device)."""

    def __init__(self, ctx: Context, rels: Sequence[Rel], edges: Sequence[Tuple[int, int, int, int]],
                 bits_per_key: int = 0, k: int = 0, block_bits: int = 0, passes: int = 0, seed: int = 0,
                 root: int = -1, workspace: Optional[torch.Tensor] = None, profile: bool = False,
                 eager: bool = False, filter_cache: "Optional[FilterCache]" = None, binary_cycles: bool = False,
                 flags: int = 0, static_workspace: bool = False, probe_grid: int = 0, probe_lds: int = 0):
        self.ctx = ctx
        self.block_bits = block_bits or 512
        self.nrels = len(rels)
        self.rels = list(rels)
        self.handle = ctypes.c_void_p()
        arr, earr, self._keep = _marshal(rels, edges)
        opts = _Opts(bits_per_key, k, block_bits, passes, seed & (2**64 - 1), root,
                     (SJ_FLAG_PROFILE if profile else 0) | (SJ_FLAG_EAGER if eager else 0) |
                     (SJ_FLAG_BINARY_CYCLES if binary_cycles else 0) | flags, probe_grid, probe_lds)
        wsb = ctypes.c_uint64()
        ctx._check(lib().sj_plan(ctx.handle, arr, len(rels), earr, len(edges), ctypes.byref(opts),
                                 ctypes.byref(self.handle), ctypes.byref(wsb)))
        self.workspace_bytes = int(wsb.value)
        if static_workspace:   # the library's static workspace: nothing is allocated
            self.workspace = None
            ctx._check(lib().sj_bind_static_workspace(self.handle))
        elif workspace is None:
            workspace = torch.empty(max(256, self.workspace_bytes), dtype=torch.uint8,
                                    device="cuda:%d" % ctx.device)
        if not static_workspace:
            self.workspace = workspace
            ctx._check(lib().sj_bind_workspace(self.handle, ctypes.c_void_p(workspace.data_ptr()),
                                               workspace.numel() * workspace.element_size()))
        self.count = None
        self.checksum = None
        self.filter_cache = None
        if filter_cache is not None:
            self.use_filter_cache(filter_cache)

    def use_filter_cache(self, cache: "Optional[FilterCache]") -> None:
        """Attach to a filter catalogue (None detaches); filters must be built again."""
        self._check(lib().sj_plan_use_filter_cache(self.handle, cache.handle if cache is not None else None))
        self.filter_cache = cache   # the catalogue outlives the attachment

    def filter_cached(self, f: int) -> int:
        """0: filter f is in the workspace, 1: reused from the catalogue, 2: built into it."""
        how = ctypes.c_int32()
        self._check(lib().sj_plan_filter_cached(self.handle, f, ctypes.byref(how)))
        return int(how.value)

    def _check(self, code):
        self.ctx._check(code)

    def build_filters(self) -> None:
        self._check(lib().sj_build_filters(self.handle))

    def sieve(self, survivors: bool = False):
        if not survivors:
            self._check(lib().sj_sieve(self.handle, None))
            return None
        out = (ctypes.c_uint64 * self.nrels)()
        self._check(lib().sj_sieve(self.handle, out))
        return [int(x) for x in out]

    def join(self) -> Tuple[int, int]:
        c, s = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(lib().sj_join(self.handle, ctypes.byref(c), ctypes.byref(s)))
        self.count, self.checksum = int(c.value), int(s.value)
        return self.count, self.checksum

    def join_async(self) -> None:
        """Enqueue the count pass; the count stays on the device (see join_wait)."""
        self._check(lib().sj_join_async(self.handle))
        self.count = None

    def result_async(self, out: torch.Tensor, mode: int = SJ_RIDS) -> torch.Tensor:
        """Enqueue the materialisation into `out` (int32 [capacity, width]); nothing is
        written if the result does not fit (join_wait reports it)."""
        cap = out.numel() // max(1, self.width(mode))
        self._check(lib().sj_result_async(self.handle, ctypes.c_void_p(out.data_ptr() if out.numel() else 0), cap,
                                          mode))
        return out

    def join_wait(self) -> Tuple[int, int, int]:
        """(count, checksum, status of the last result_async) after waiting for the stream."""
        c, k, st = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int32()
        self._check(lib().sj_join_wait(self.handle, ctypes.byref(c), ctypes.byref(k), ctypes.byref(st)))
        self.count, self.checksum = int(c.value), int(k.value)
        return self.count, self.checksum, int(st.value)

    def result(self, out: Optional[torch.Tensor] = None, mode: int = SJ_RIDS) -> torch.Tensor:
        """The result tuples: int32 [count, nrels] row ids (SJ_RIDS) or [count, width]
        projected values (SJ_VALUES, see set_projection)."""
        if self.count is None:
            raise SjError(SJ_ERR_STATE, "call join() first")
        w = self.width(mode)
        if out is None:
            out = torch.empty((self.count, w), dtype=torch.int32, device="cuda:%d" % self.ctx.device)
        cap = out.numel() // max(1, w)
        self._check(lib().sj_result(self.handle, ctypes.c_void_p(out.data_ptr() if out.numel() else 0), cap, mode))
        return out

    def set_projection(self, cols: Sequence[Tuple[int, int]]) -> None:
        """Columns SJ_VALUES writes: (relation, column) pairs ([] = every column of every relation)."""
        flat = (ctypes.c_int32 * max(1, 2 * len(cols)))(*[int(x) for rc in cols for x in rc])
        self._check(lib().sj_plan_set_projection(self.handle, flat, len(cols)))

    def width(self, mode: int = SJ_RIDS) -> int:
        w = ctypes.c_int32()
        self._check(lib().sj_plan_footprint(self.handle, mode, None, None, ctypes.byref(w)))
        return int(w.value)

    def footprint(self, mode: int = SJ_RIDS) -> dict:
        """Workspace bytes, result width and (once counted) result bytes in `mode`."""
        ws, rb, w = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int32()
        code = lib().sj_plan_footprint(self.handle, mode, ctypes.byref(ws), ctypes.byref(rb), ctypes.byref(w))
        if code not in (SJ_OK, SJ_ERR_STATE):
            self._check(code)
        return {"workspace_bytes": int(ws.value), "width": int(w.value),
                "result_bytes": int(rb.value) if code == SJ_OK else None}

    def run(self) -> Tuple[int, int, torch.Tensor]:
        self.build_filters()
        self.sieve()
        c, s = self.join()
        return c, s, self.result()

    # ---- introspection
    def filter_count(self) -> int:
        n = ctypes.c_int32()
        self._check(lib().sj_filter_count(self.handle, ctypes.byref(n)))
        return int(n.value)

    def filter_desc(self, f: int, nblocks: bool = True) -> dict:
        """Filter f's identity; its size in blocks (after build_filters) unless nblocks=False."""
        kind, index, rel, col = (ctypes.c_int32() for _ in range(4))
        nb = ctypes.c_uint32()
        self._check(lib().sj_filter_desc(self.handle, f, ctypes.byref(kind), ctypes.byref(index),
                                         ctypes.byref(rel), ctypes.byref(col),
                                         ctypes.byref(nb) if nblocks else None))
        d = dict(kind=int(kind.value), index=int(index.value), src_rel=int(rel.value), src_col=int(col.value))
        if nblocks:
            d["nblocks"] = int(nb.value)
        return d

    def filter_words(self, f: int) -> torch.Tensor:
        d = self.filter_desc(f)
        out = torch.empty(d["nblocks"] * self.block_bits // 32, dtype=torch.int32, device="cuda:%d" % self.ctx.device)
        self._check(lib().sj_filter_copy(self.handle, f, ctypes.c_void_p(out.data_ptr()), out.numel()))
        return out

    def _filter_update(self, fn, f: int, keys: torch.Tensor):
        if keys.dtype != torch.int32 or keys.dim() != 1 or not keys.is_contiguous():
            raise ValueError("keys must be a contiguous 1-D int32 tensor")
        flags = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        cnt = ctypes.c_uint64()
        self._check(fn(self.handle, f, ctypes.c_void_p(keys.data_ptr()), keys.numel(),
                       ctypes.c_void_p(flags.data_ptr()), ctypes.byref(cnt)))
        return flags.bool(), int(cnt.value)

    def filter_probe(self, f: int, keys: torch.Tensor):
        """(contained bool tensor, number of keys filter f does not contain)."""
        return self._filter_update(lib().sj_filter_probe, f, keys)

    def filter_insert(self, f: int, keys: torch.Tensor):
        """Insert keys into filter f in place: (contained before the call, number inserted)."""
        return self._filter_update(lib().sj_filter_insert, f, keys)

    def propagate(self, rel: int, cols: Sequence[torch.Tensor]) -> List[int]:
        """Insert new rows of relation `rel` (int32 device columns, the relation's full
        column set) into the backward filters from `rel` toward the root (Section 2.4);
        returns, per relation, how many keys its filter did not hold."""
        n = cols[0].numel() if cols else 0
        for c in cols:
            if c.dtype != torch.int32 or c.dim() != 1 or c.numel() != n or not c.is_contiguous():
                raise ValueError("columns must be contiguous 1-D int32 tensors of equal length")
        nb = ctypes.c_uint64()
        self._check(lib().sj_filter_propagate_scratch(self.handle, rel, n, ctypes.byref(nb)))
        scratch = torch.empty(max(256, nb.value), dtype=torch.uint8, device="cuda:%d" % self.ctx.device)
        ptrs = (ctypes.c_void_p * max(1, len(cols)))(*[c.data_ptr() for c in cols])
        out = (ctypes.c_uint64 * self.nrels)()
        self._check(lib().sj_filter_propagate(self.handle, rel, ptrs, n, ctypes.c_void_p(scratch.data_ptr()),
                                              scratch.numel(), out))
        return [int(x) for x in out]

    def counting_filter(self, f: int) -> "CountingFilter":
        """The counting twin of filter f (Section 2.4), built from the keys f was built from."""
        return CountingFilter(self, f)

    def survivors(self, rel: int) -> torch.Tensor:
        n = ctypes.c_uint64()
        self._check(lib().sj_survivors_copy(self.handle, rel, None, 0, ctypes.byref(n)))
        out = torch.empty(int(n.value), dtype=torch.int32, device="cuda:%d" % self.ctx.device)
        if out.numel():
            self._check(lib().sj_survivors_copy(self.handle, rel, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                                ctypes.byref(n)))
        return out

    def profile(self, reset: bool = False) -> List[dict]:
        """Per launch-group event timings (plans made with profile=True)."""
        self._check(lib().sj_profile_collect(self.handle))
        n = ctypes.c_int32()
        self._check(lib().sj_profile_count(self.handle, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            lab, ms, cnt, by = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64()
            self._check(lib().sj_profile_entry(self.handle, i, ctypes.byref(lab), ctypes.byref(ms),
                                               ctypes.byref(cnt), ctypes.byref(by)))
            out.append(dict(label=lab.value.decode(), total_ms=ms.value, launches=int(cnt.value),
                            alg_bytes=int(by.value)))
        if reset:
            self._check(lib().sj_profile_reset(self.handle))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.sj_plan_destroy(h)
            self.handle = None


class CountingFilter:
    """sj_cfilter: 4-bit counters twinning a plan's filter; insert/delete/probe/export."""

    def __init__(self, plan: Plan, f: int):
        self.plan = plan
        self.f = f
        nblocks = plan.filter_desc(f)["nblocks"]
        self.counts = torch.empty(nblocks * plan.block_bits // 2 + 256, dtype=torch.uint8,
                                  device="cuda:%d" % plan.ctx.device)
        self.nwords = nblocks * plan.block_bits // 32
        self.handle = ctypes.c_void_p()
        plan._check(lib().sj_plan_cfilter(plan.handle, f, ctypes.c_void_p(self.counts.data_ptr()),
                                          self.counts.numel(), ctypes.byref(self.handle)))

    def _keys(self, keys: torch.Tensor) -> torch.Tensor:
        if keys.dtype != torch.int32 or keys.dim() != 1 or not keys.is_contiguous():
            raise ValueError("keys must be a contiguous 1-D int32 tensor")
        return keys

    def insert(self, keys: torch.Tensor) -> None:
        k = self._keys(keys)
        self.plan._check(lib().sj_cfilter_update(self.handle, ctypes.c_void_p(k.data_ptr()), k.numel(), 1))

    def delete(self, keys: torch.Tensor) -> None:
        k = self._keys(keys)
        self.plan._check(lib().sj_cfilter_update(self.handle, ctypes.c_void_p(k.data_ptr()), k.numel(), -1))

    def probe(self, keys: torch.Tensor):
        k = self._keys(keys)
        flags = torch.empty(k.numel(), dtype=torch.uint8, device=k.device)
        miss = ctypes.c_uint64()
        self.plan._check(lib().sj_cfilter_probe(self.handle, ctypes.c_void_p(k.data_ptr()), k.numel(),
                                                ctypes.c_void_p(flags.data_ptr()), ctypes.byref(miss)))
        return flags.bool(), int(miss.value)

    def export(self) -> torch.Tensor:
        out = torch.empty(self.nwords, dtype=torch.int32, device=self.counts.device)
        self.plan._check(lib().sj_cfilter_export(self.handle, ctypes.c_void_p(out.data_ptr()), out.numel()))
        return out

    def apply(self) -> None:
        """Write the exported bits over the plan's filter."""
        self.plan._check(lib().sj_cfilter_apply(self.handle, self.plan.handle, self.f))

    def counters(self) -> torch.Tensor:
        """The counter words (uint32 view, 8 counters of 4 bits each per word)."""
        return self.counts[: self.nwords * 16].view(torch.int32)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.sj_cfilter_destroy(h)
            self.handle = None


class Batch:
    """sj_batch: the whole query of every plan (all made on `ctx`) recorded into one graph
    and replayed by submit(); each plan's count, checksum and status then come from its
    join_wait(). The plans are kept alive by the batch."""

    def __init__(self, ctx: Context, plans: Sequence[Plan]):
        self.ctx = ctx
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        self.handle = ctypes.c_void_p()
        ctx._check(lib().sj_batch_create(ctx.handle, arr, len(self.plans), ctypes.byref(self.handle)))

    def submit(self, outs: Optional[Sequence[Optional[torch.Tensor]]] = None, mode: int = SJ_RIDS) -> None:
        """Enqueue every plan's query; outs[i] (int32 [capacity, width] or None) receives
        plan i's tuples."""
        n = len(self.plans)
        if outs is None:
            self.ctx._check(lib().sj_batch_submit(self.handle, None, None, mode))
            return
        ptrs = (ctypes.c_void_p * n)(*[(o.data_ptr() if o is not None and o.numel() else None) for o in outs])
        caps = (ctypes.c_uint64 * n)(*[(o.numel() // max(1, p.width(mode)) if o is not None else 0)
                                       for o, p in zip(outs, self.plans)])
        self.ctx._check(lib().sj_batch_submit(self.handle, ptrs, caps, mode))
        for p in self.plans:
            p.count = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.sj_batch_destroy(h)
            self.handle = None


class FilterCache:
    """sj_fcache over a torch uint8 arena: backward filters kept resident across queries.

    Plans attach with Plan(..., filter_cache=c) or plan.use_filter_cache(c); a server
    with server.use_filter_cache(c). Attached plans and servers keep the catalogue
    alive."""

    def __init__(self, arena_bytes: int, device: int = 0, arena: Optional[torch.Tensor] = None):
        self.device = device
        self.arena = arena if arena is not None else torch.empty(arena_bytes, dtype=torch.uint8,
                                                                  device="cuda:%d" % device)
        self.handle = ctypes.c_void_p()
        torch.cuda.synchronize(device)
        code = lib().sj_fcache_create(device, ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                      ctypes.byref(self.handle))
        if code != SJ_OK:
            raise SjError(code, "sj_fcache_create")

    def stats(self) -> dict:
        i = _FcInfo()
        code = lib().sj_fcache_stats(self.handle, ctypes.byref(i))
        if code != SJ_OK:
            raise SjError(code, "sj_fcache_stats")
        return {n: int(getattr(i, n)) for n, _ in _FcInfo._fields_}

    def invalidate(self, column) -> None:
        """Drop the entries built from `column` (a device tensor or pointer) after an in-place change."""
        ptr = column.data_ptr() if isinstance(column, torch.Tensor) else int(column)
        code = lib().sj_fcache_invalidate(self.handle, ctypes.c_void_p(ptr))
        if code != SJ_OK:
            raise SjError(code, "sj_fcache_invalidate")

    def clear(self) -> None:
        code = lib().sj_fcache_clear(self.handle)
        if code != SJ_OK:
            raise SjError(code, "sj_fcache_clear")

    def close(self) -> None:
        if self.handle and _lib is not None:
            code = _lib.sj_fcache_destroy(self.handle)
            if code != SJ_OK:
                raise SjError(code, "sj_fcache_destroy: plans still hold entries")
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            if _lib.sj_fcache_destroy(self.handle) == SJ_OK:
                self.handle = None


class Server:
    """sj_server over a torch uint8 arena on `device` with `slots` workers.

    submit() queues a query and returns its ticket; info(ticket, wait) returns its state
    as a dict; result(ticket) is a zero-copy int32 [count, nrels] view of the arena;
    release(ticket) frees it. Input tensors are kept alive until release."""

    def __init__(self, arena_bytes: int, slots: int = 4, device: int = 0, arena: Optional[torch.Tensor] = None):
        self.device = device
        self.arena = arena if arena is not None else torch.empty(arena_bytes, dtype=torch.uint8,
                                                                  device="cuda:%d" % device)
        self.handle = ctypes.c_void_p()
        self._alive = {}
        self.filter_cache = None
        torch.cuda.synchronize(device)   # the arena's allocation is complete before workers use it
        code = lib().sj_server_create(device, ctypes.c_void_p(self.arena.data_ptr()),
                                      self.arena.numel(), slots, ctypes.byref(self.handle))
        if code != SJ_OK:
            raise SjError(code, "sj_server_create")

    def submit(self, rels: Sequence[Rel], edges: Sequence[Tuple[int, int, int, int]], bits_per_key: int = 0,
               k: int = 0, block_bits: int = 0, passes: int = 0, seed: int = 0, root: int = -1,
               count_only: bool = False, values: bool = False, flags: int = 0, probe_grid: int = 0,
               probe_lds: int = 0) -> int:
        """Queue a query; its result is row ids (default), values (all columns of every
        relation, relation order) or the count only."""
        arr, earr, keep = _marshal(rels, edges)
        opts = _Opts(bits_per_key, k, block_bits, passes, seed & (2**64 - 1), root, flags, probe_grid, probe_lds)
        t = ctypes.c_uint64()
        mode = SJ_RESULT_COUNT if count_only else (SJ_RESULT_VALUES if values else SJ_RESULT_TUPLES)
        code = lib().sj_server_submit(self.handle, arr, len(rels), earr, len(edges), ctypes.byref(opts),
                                      mode, ctypes.byref(t))
        if code != SJ_OK:
            raise SjError(code, (lib().sj_server_last_error(self.handle) or b"").decode())
        width = sum(len(r.cols) for r in rels) if values else len(rels)
        self._alive[int(t.value)] = (list(rels), width, keep)
        return int(t.value)

    def info(self, ticket: int, wait: bool = False) -> dict:
        q = _QueryInfo()
        code = lib().sj_server_query(self.handle, ticket, 1 if wait else 0, ctypes.byref(q))
        if code != SJ_OK:
            raise SjError(code, "unknown ticket %d" % ticket)
        return {"state": q.state, "status": q.status, "count": int(q.count), "checksum": int(q.checksum),
                "result_offset": int(q.result_offset), "workspace_bytes": int(q.workspace_bytes),
                "t_submit_ns": int(q.t_submit_ns), "t_admit_ns": int(q.t_admit_ns), "t_done_ns": int(q.t_done_ns),
                "slot": int(q.slot), "requeues": int(q.requeues), "error": q.error.decode()}

    def result(self, ticket: int) -> torch.Tensor:
        q = self.info(ticket, wait=True)
        if q["state"] != SJ_QUERY_DONE:
            raise SjError(q["status"], q["error"])
        width = self._alive[ticket][1]
        n = q["count"] * width
        if n == 0:
            return torch.empty((0, width), dtype=torch.int32, device=self.arena.device)
        off = q["result_offset"]
        return self.arena[off: off + 4 * n].view(torch.int32).view(q["count"], width)

    def use_filter_cache(self, cache: Optional[FilterCache]) -> None:
        """Attach every query admitted from now on to `cache` (None: none)."""
        code = lib().sj_server_use_filter_cache(self.handle, cache.handle if cache is not None else None)
        if code != SJ_OK:
            raise SjError(code, "sj_server_use_filter_cache")
        self.filter_cache = cache

    def release(self, ticket: int) -> None:
        code = lib().sj_server_release(self.handle, ticket)
        if code != SJ_OK:
            raise SjError(code, "release of ticket %d" % ticket)
        self._alive.pop(ticket, None)

    def stats(self) -> dict:
        used, peak = ctypes.c_uint64(), ctypes.c_uint64()
        queued, running = ctypes.c_int32(), ctypes.c_int32()
        lib().sj_server_stats(self.handle, ctypes.byref(used), ctypes.byref(peak), ctypes.byref(queued),
                              ctypes.byref(running))
        return {"arena_used": int(used.value), "arena_peak": int(peak.value), "queued": int(queued.value),
                "running": int(running.value)}

    def close(self) -> None:
        if self.handle and _lib is not None:
            _lib.sj_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()
