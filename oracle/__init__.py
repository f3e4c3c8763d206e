"""CPU oracle for the SieveJoin hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never loads it and shares
no code with it.

What it computes (arXiv 2308.16370):

* ``hash_join``  -- the exact multi-way join result by a plain left-deep binary
  hash-join plan with no filters (the enumeration phase of Section 2.2 with the
  pruning switched off), as sorted row-id tuples plus count and checksum.
* ``join_tree_dp`` -- count and checksum of an acyclic join by the sum-product
  recursion over the join tree (Yannakakis-style, the paper's reference list
  includes it); independent of ``hash_join``.
* ``bf_*``       -- the blocked Bloom filter (Section 2.1 step 1, Bloom's bit vector
  in its cache-blocked form) under the hash/bit-pattern reading stated in
  ``oracle.c``.
* ``project``    -- value tuples from row-id tuples (the join result as values, each
  row id replaced by its row's values in the chosen columns).
* ``cf_update`` / ``cf_export`` / ``propagate`` -- update maintenance (Section 2.4):
  counting twins of the blocked filters (inserts and deletes) and the propagation of
  inserted tuples toward the root.
* ``triangle_cycles`` -- count and checksum of the directed 3-cycle query by
  adjacency intersection (a textbook triangle count), independent of ``hash_join``.
* ``clique4``    -- count and checksum of the 4-clique query (Section 3.1.3) by a
  generic join over its four variables, independent of ``hash_join``.
* ``sieve``      -- the pruning phase (Section 2.2): one backward pass from the
  right-most relation to the root, each relation probed by the filters of the
  relations after it and building the filter on its own join attribute from its
  survivors; the closing-edge filter of cyclic queries (Section 2.3); and the
  optional forward pass (the dotted arrow of Fig. 2) that sieves the relations on
  the right with filters of their already-pruned left neighbours.

The checksum of a result is sum over tuples of prod_i (mix64((i << 32) | rid_i) | 1)
modulo 2^64, with mix64 the SplitMix64 output function.

Every function here is pinned by tests/test_oracle_*.py against brute force, closed
forms, the paper's worked example and the filter's probability laws.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

U64 = np.uint64
MASK64 = (1 << 64) - 1


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            c_u32p = ctypes.POINTER(ctypes.c_uint32)
            L.orc_fmix32.argtypes = [ctypes.c_uint32]
            L.orc_fmix32.restype = ctypes.c_uint32
            L.orc_mix64.argtypes = [ctypes.c_uint64]
            L.orc_mix64.restype = ctypes.c_uint64
            L.orc_chk_factor.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
            L.orc_chk_factor.restype = ctypes.c_uint64
            L.orc_bf_nblocks.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
            L.orc_bf_nblocks.restype = ctypes.c_uint64
            L.orc_bf_pattern.argtypes = [ctypes.c_int32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_uint32, c_u32p]
            L.orc_bf_pattern.restype = ctypes.c_uint32
            L.orc_bf_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_uint32]
            L.orc_bf_build.restype = None
            L.orc_bf_probe.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                       ctypes.c_void_p]
            L.orc_bf_probe.restype = None
            ip = ctypes.POINTER(ctypes.c_int)
            L.orc_hash_join.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int, ip, ip, ip, ip, ctypes.c_int,
                                        ip, ip, ip, ip, ip]
            L.orc_hash_join.restype = ctypes.c_void_p
            L.orc_result_count.argtypes = [ctypes.c_void_p]
            L.orc_result_count.restype = ctypes.c_int64
            L.orc_triangle_cycles.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)]
            L.orc_triangle_cycles.restype = ctypes.c_int
            L.orc_clique4.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)]
            L.orc_clique4.restype = ctypes.c_int
            L.orc_result_checksum.argtypes = [ctypes.c_void_p]
            L.orc_result_checksum.restype = ctypes.c_uint64
            L.orc_result_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            L.orc_result_copy.restype = None
            L.orc_result_free.argtypes = [ctypes.c_void_p]
            L.orc_result_free.restype = None
            _lib = L
    return _lib


# ---------------------------------------------------------------- mixers / checksum

def fmix32(x: int) -> int:
    return int(lib().orc_fmix32(x & 0xFFFFFFFF))


def mix64(x: int) -> int:
    return int(lib().orc_mix64(x & MASK64))


def mix64_np(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.astype(U64, copy=True)
    z ^= z >> U64(30)
    z *= U64(0xBF58476D1CE4E5B9)
    z ^= z >> U64(27)
    z *= U64(0x94D049BB133111EB)
    z ^= z >> U64(31)
    return z


def chk_factor_np(rel: int, rids: np.ndarray) -> np.ndarray:
    """mix64((rel << 32) | rid) | 1 for every rid."""
    z = (U64(rel) << U64(32)) | rids.astype(U64)
    return mix64_np(z) | U64(1)


def filter_seed(seed: int) -> int:
    """The 32-bit filter hash seed derived from the 64-bit user seed."""
    return mix64(seed) & 0xFFFFFFFF


# ---------------------------------------------------------------- Bloom filter

def log2_block(block_bits: int) -> int:
    lb = int(block_bits).bit_length() - 1
    if block_bits not in (256, 512, 1024):
        raise ValueError("block_bits must be 256, 512 or 1024")
    return lb


def bf_nblocks(n: int, bits_per_key: int, block_bits: int = 512) -> int:
    return int(lib().orc_bf_nblocks(int(n), int(bits_per_key), log2_block(block_bits)))


def bf_pattern(key: int, nblocks: int, k: int, block_bits: int, seed32: int) -> Tuple[int, List[int]]:
    pos = (ctypes.c_uint32 * 64)()
    b = lib().orc_bf_pattern(int(np.int32(key)), nblocks, k, log2_block(block_bits), seed32, pos)
    return int(b), [int(pos[i]) for i in range(k)]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def bf_build(keys: np.ndarray, rows: Optional[np.ndarray], nblocks: int, k: int,
             block_bits: int, seed32: int) -> np.ndarray:
    """Filter words (uint32, nblocks * block_bits/32) holding keys[rows] (or all keys)."""
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    words = np.zeros(nblocks * (block_bits // 32), dtype=np.uint32)
    n = keys.shape[0] if rows is None else rows.shape[0]
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.uint32)
    lib().orc_bf_build(_ptr(keys), _ptr(rows), n, _ptr(words), nblocks, k, log2_block(block_bits), seed32)
    return words


def bf_probe(words: np.ndarray, keys: np.ndarray, rows: Optional[np.ndarray], nblocks: int, k: int,
             block_bits: int, seed32: int) -> np.ndarray:
    """Boolean array: does the filter report keys[rows[i]] (or keys[i]) present."""
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    n = keys.shape[0] if rows is None else rows.shape[0]
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.uint32)
    out = np.zeros(n, dtype=np.uint8)
    lib().orc_bf_probe(_ptr(keys), _ptr(rows), n, _ptr(np.ascontiguousarray(words, dtype=np.uint32)),
                       nblocks, k, log2_block(block_bits), seed32, _ptr(out))
    return out.astype(bool)


def bf_insert(words: np.ndarray, keys: np.ndarray, nblocks: int, k: int, block_bits: int,
              seed32: int) -> Tuple[np.ndarray, np.ndarray]:
    """Insert keys into a built filter (Section 2.4): which keys it contained before
    (those change nothing), and the filter with every key's pattern bits set (the
    block count is kept). Setting a contained key's bits again changes nothing, so the
    new words are the old ones OR the words of a filter of the keys alone."""
    contained = bf_probe(words, keys, None, nblocks, k, block_bits, seed32)
    new = np.asarray(words, dtype=np.uint32) | bf_build(keys, None, nblocks, k, block_bits, seed32)
    return new, contained


# ---------------------------------------------------------------- updates (Section 2.4)

def cf_update(counts: np.ndarray, keys: np.ndarray, sign: int, nblocks: int, k: int, block_bits: int,
              seed32: int) -> np.ndarray:
    """Counting filter (Section 2.4: a counter per position makes deletions possible):
    counts is uint8 [nblocks, block_bits], one counter per bit position of the blocked
    filter. Each key adds (sign +1) or removes (sign -1) one at each of its k pattern
    positions (a position repeated in the pattern counts twice). Counters saturate at 15
    and a saturated counter is never decremented; a counter at 0 is not decremented."""
    c = counts.copy()
    for key in np.asarray(keys, dtype=np.int32).tolist():
        b, pos = bf_pattern(key, nblocks, k, block_bits, seed32)
        for p in pos:
            v = int(c[b, p])
            if v == 15:
                continue
            if sign > 0:
                c[b, p] = v + 1
            elif v > 0:
                c[b, p] = v - 1
    return c


def cf_export(counts: np.ndarray) -> np.ndarray:
    """The plain filter words of a counting filter: bit p of block b is set iff its
    counter is nonzero (word b * B/32 + p // 32, bit p % 32)."""
    nb, B = counts.shape
    bits = (counts > 0).astype(np.uint64).reshape(nb * B // 32, 32)
    return (bits << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)


def propagate(query, filters: Dict[int, Tuple[np.ndarray, int]], rel: int, new_cols: Sequence[np.ndarray],
              k: int, block_bits: int, seed32: int, root: Optional[int] = None):
    """Section 2.4: new tuples of relation `rel` (columns new_cols) go into the backward
    filters from rel toward the root. filters maps each non-root relation j to its
    backward filter (words, nblocks) on j's key toward its parent. The new rows that
    pass rel's predicate and its children's filters insert their key into rel's filter;
    a key the filter did not contain leads to the parent: its rows whose key toward the
    child is among those keys, that pass its predicate and its other children's filters,
    insert their own key into its filter, and so on until the root (which has no
    backward filter). Returns (new filters, keys not contained per relation, counted
    with multiplicity)."""
    root = query.root if root is None else root
    t = JoinTree(len(query.rels), query.edges, root)
    F = {j: (np.asarray(w, dtype=np.uint32).copy(), nb) for j, (w, nb) in filters.items()}
    inserted = [0] * len(query.rels)
    if rel == root or len(new_cols) == 0 or new_cols[0].shape[0] == 0:
        return F, inserted
    j, child, missing = rel, None, None
    while True:
        R = query.rels[j]
        cols = [np.asarray(c, dtype=np.int32) for c in (new_cols if child is None else R.cols)]
        ok = np.ones(cols[0].shape[0], dtype=bool)
        if child is not None:
            ok &= np.isin(cols[t.pcol[child]], missing)
        if R.pred is not None:
            pc, lo, hi = R.pred
            ok &= (cols[pc].astype(np.int64) >= lo) & (cols[pc].astype(np.int64) < hi)
        for c in t.children[j]:
            if c == child:
                continue
            w, nb = F[c]
            ok &= bf_probe(w, cols[t.pcol[c]], None, nb, k, block_bits, seed32)
        keys = cols[t.mycol[j]][ok]
        if keys.shape[0] == 0:
            break
        w, nb = F[j]
        neww, contained = bf_insert(w, keys, nb, k, block_bits, seed32)
        F[j] = (neww, nb)
        inserted[j] = int((~contained).sum())
        par = t.parent[j]
        if inserted[j] == 0 or par == root:
            break
        missing = np.unique(keys[~contained])
        child, j = j, par
    return F, inserted


# ---------------------------------------------------------------- join graph

class JoinTree:
    """Root, spanning tree and closing edges of a join graph.

    The tree is found by depth-first search from the root that follows each
    relation's edges in input order; edges not taken by the search are closing
    edges. For a closing edge, ``u`` is the end visited first (preorder) and ``v``
    the other.
    """

    def __init__(self, nrels: int, edges: Sequence[Tuple[int, int, int, int]], root: int = 0):
        self.n = nrels
        self.root = root
        adj: List[List[Tuple[int, int, int, int]]] = [[] for _ in range(nrels)]
        for ei, (ra, ca, rb, cb) in enumerate(edges):
            if not (0 <= ra < nrels and 0 <= rb < nrels) or ra == rb:
                raise ValueError("bad edge %r" % (edges[ei],))
            adj[ra].append((ei, rb, ca, cb))
            adj[rb].append((ei, ra, cb, ca))
        self.parent = [-1] * nrels
        self.pcol = [-1] * nrels     # column of the parent on the tree edge to this relation
        self.mycol = [-1] * nrels    # this relation's column on its tree edge to the parent
        self.children: List[List[int]] = [[] for _ in range(nrels)]
        self.preorder: List[int] = []
        tree_edges = set()
        seen = [False] * nrels

        def dfs(u):
            seen[u] = True
            self.preorder.append(u)
            for ei, v, cu, cv in adj[u]:
                if not seen[v]:
                    tree_edges.add(ei)
                    self.parent[v], self.pcol[v], self.mycol[v] = u, cu, cv
                    self.children[u].append(v)
                    dfs(v)

        dfs(root)
        if not all(seen):
            raise ValueError("join graph is not connected")
        pre = {r: i for i, r in enumerate(self.preorder)}
        self.closing = []            # (u, col_u, v, col_v) in input order
        for ei, (ra, ca, rb, cb) in enumerate(edges):
            if ei in tree_edges:
                continue
            if pre[ra] < pre[rb]:
                self.closing.append((ra, ca, rb, cb))
            else:
                self.closing.append((rb, cb, ra, ca))
        self.postorder: List[int] = []

        def post(u):
            for c in self.children[u]:
                post(c)
            self.postorder.append(u)

        post(root)


def eligible(rel) -> np.ndarray:
    """Ascending row ids that pass the relation's predicate lo <= v < hi."""
    n = rel.nrows
    if rel.pred is None:
        return np.arange(n, dtype=np.uint32)
    c, lo, hi = rel.pred
    v = rel.cols[c].astype(np.int64)
    return np.nonzero((v >= lo) & (v < hi))[0].astype(np.uint32)


# ---------------------------------------------------------------- hash join

def hash_join(query, root: Optional[int] = None):
    """Sorted result row-id tuples (uint32 [count, nrels]), count, checksum."""
    root = query.root if root is None else root
    n = len(query.rels)
    t = JoinTree(n, query.edges, root)
    maxcols = max(len(r.cols) for r in query.rels)
    keep = []
    colptrs = (ctypes.c_void_p * (n * maxcols))()
    for r, rel in enumerate(query.rels):
        for c, col in enumerate(rel.cols):
            a = np.ascontiguousarray(col, dtype=np.int32)
            keep.append(a)
            colptrs[r * maxcols + c] = a.ctypes.data
    sels = [eligible(rel) for rel in query.rels]
    selptrs = (ctypes.c_void_p * n)(*[s.ctypes.data if s.size else None for s in sels])
    nsel = (ctypes.c_int64 * n)(*[int(s.shape[0]) for s in sels])
    order = t.preorder
    steps = order[1:]
    IA = ctypes.c_int * max(1, n - 1)
    child = IA(*steps)
    ccol = IA(*[t.mycol[c] for c in steps])
    par = IA(*[t.parent[c] for c in steps])
    pcol = IA(*[t.pcol[c] for c in steps])
    pos = {r: i for i, r in enumerate(order)}
    nc = len(t.closing)
    CA = ctypes.c_int * max(1, nc)
    after = [max(pos[u], pos[v]) - 1 for (u, _, v, _) in t.closing]
    res = lib().orc_hash_join(n, maxcols, colptrs, selptrs, nsel, root, child, ccol, par, pcol, nc,
                              CA(*[c[0] for c in t.closing]), CA(*[c[1] for c in t.closing]),
                              CA(*[c[2] for c in t.closing]), CA(*[c[3] for c in t.closing]),
                              CA(*after))
    if not res:
        raise MemoryError("oracle hash join ran out of memory")
    try:
        cnt = int(lib().orc_result_count(res))
        chk = int(lib().orc_result_checksum(res))
        out = np.empty((cnt, n), dtype=np.uint32)
        lib().orc_result_copy(res, out.ctypes.data_as(ctypes.c_void_p))
    finally:
        lib().orc_result_free(res)
    return out, cnt, chk


def triangle_cycles(src: np.ndarray, dst: np.ndarray, e1: Optional[Tuple[np.ndarray, np.ndarray]] = None
                    ) -> Tuple[int, int]:
    """Count and checksum of E1 join E2 join E3 on E1.dst = E2.src, E2.dst = E3.src,
    E3.dst = E1.src with E2 = E3 = the edge list (src, dst) (the 3-cycle query,
    Section 2.3), by adjacency intersection: for every E1 edge a -> b, the out-edges
    of b and the in-edges of a that meet in one vertex. E1 is the same edge list, or
    ``e1 = (e1_src, e1_dst)`` (for instance a sample of its rows, numbered 0..m-1).
    Independent of ``hash_join``."""
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    if e1 is None:
        s1, d1 = s, d
    else:
        s1 = np.ascontiguousarray(e1[0], dtype=np.int32)
        d1 = np.ascontiguousarray(e1[1], dtype=np.int32)
        if s1.shape != d1.shape:
            raise ValueError("e1 columns differ in length")
    cnt, chk = ctypes.c_int64(), ctypes.c_uint64()
    if lib().orc_triangle_cycles(s.shape[0], _ptr(s), _ptr(d), s1.shape[0], _ptr(s1), _ptr(d1), ctypes.byref(cnt),
                                 ctypes.byref(chk)) != 0:
        raise MemoryError("orc_triangle_cycles")
    return int(cnt.value), int(chk.value)



# ---------------------------------------------------------------- 4-cliques

def clique4_roles(query, root: Optional[int] = None):
    """The variables of a 4-clique query, or None if the query is not one.

    Join edges put (relation, column) pairs into variables (classes of columns that
    must be equal). A 4-clique query has six relations and four variables; every
    relation joins on exactly two columns, of two different variables, and the six
    relations hold the six different pairs. The root's two variables are a and b (its
    lower join column first); c and d are the other two, ordered by their first
    (relation, column). Returns [(relation, column of x, column of y)] for the pairs
    (x, y) = ab, ac, ad, bc, bd, cd."""
    root = query.root if root is None else root
    if len(query.rels) != 6:
        return None
    up = {}

    def find(u):
        while up.setdefault(u, u) != u:
            u = up[u]
        return u

    for a, ca, b, cb in query.edges:
        ra, rb = find((a, ca)), find((b, cb))
        if ra != rb:
            up[max(ra, rb)] = min(ra, rb)
    used = {}
    for a, ca, b, cb in query.edges:
        used.setdefault(a, set()).add(ca)
        used.setdefault(b, set()).add(cb)
    if sorted(used) != list(range(6)) or any(len(c) != 2 for c in used.values()):
        return None
    var = {u: find(u) for u in list(up)}
    classes = sorted(set(var.values()))
    if len(classes) != 4:
        return None
    pair_rel = {}
    for r in range(6):
        c0, c1 = sorted(used[r])
        v0, v1 = var[(r, c0)], var[(r, c1)]
        key = frozenset((v0, v1))
        if v0 == v1 or key in pair_rel:
            return None
        pair_rel[key] = (r, {v0: c0, v1: c1})
    c0, c1 = sorted(used[root])
    A, B = var[(root, c0)], var[(root, c1)]
    C, D = [v for v in classes if v not in (A, B)]
    out = []
    for x, y in ((A, B), (A, C), (A, D), (B, C), (B, D), (C, D)):
        r, cols = pair_rel[frozenset((x, y))]
        out.append((r, cols[x], cols[y]))
    return out


def clique4(query, root: Optional[int] = None) -> Tuple[int, int]:
    """Count and checksum of a 4-clique query (Section 3.1.3) by a generic join over
    its variables (oracle.c, section 5), each relation's rows restricted to its
    predicate. Independent of ``hash_join``, which enumerates the same result along a
    spanning tree and checks the closing edges."""
    roles = clique4_roles(query, root)
    if roles is None:
        raise ValueError("not a 4-clique query")
    keep = []
    n = (ctypes.c_int64 * 6)()
    xs = (ctypes.c_void_p * 6)()
    ys = (ctypes.c_void_p * 6)()
    ids = (ctypes.c_void_p * 6)()
    rel = (ctypes.c_uint32 * 6)()
    for i, (r, cx, cy) in enumerate(roles):
        R = query.rels[r]
        sel = eligible(R)
        x = np.ascontiguousarray(np.asarray(R.cols[cx], dtype=np.int32)[sel])
        y = np.ascontiguousarray(np.asarray(R.cols[cy], dtype=np.int32)[sel])
        sid = np.ascontiguousarray(sel, dtype=np.uint32)
        keep += [x, y, sid]
        n[i] = sel.shape[0]
        xs[i], ys[i], ids[i] = _ptr(x), _ptr(y), _ptr(sid)
        rel[i] = r
    cnt, chk = ctypes.c_int64(), ctypes.c_uint64()
    if lib().orc_clique4(n, xs, ys, ids, rel, ctypes.byref(cnt), ctypes.byref(chk)) != 0:
        raise MemoryError("orc_clique4")
    return int(cnt.value), int(chk.value)

def default_projection(query) -> List[Tuple[int, int]]:
    """Every column of every relation, relations in index order."""
    return [(r, c) for r, rel in enumerate(query.rels) for c in range(len(rel.cols))]


def project(query, tuples: np.ndarray, cols: Optional[Sequence[Tuple[int, int]]] = None) -> np.ndarray:
    """Value tuples of a [count, nrels] row-id result: output column q holds column
    cols[q][1] of relation cols[q][0] at the tuple's row of that relation (the join
    result of Section 2.2 as values rather than row ids; default: every column of every
    relation, relations in index order). int32 [count, len(cols)]."""
    cols = default_projection(query) if cols is None else list(cols)
    out = np.empty((tuples.shape[0], len(cols)), dtype=np.int32)
    for q, (r, c) in enumerate(cols):
        out[:, q] = np.asarray(query.rels[r].cols[c], dtype=np.int32)[tuples[:, r].astype(np.int64)]
    return out


def checksum_of(tuples: np.ndarray) -> int:
    """Checksum of a [count, nrels] row-id tuple array."""
    if tuples.shape[0] == 0:
        return 0
    f = np.ones(tuples.shape[0], dtype=U64)
    for r in range(tuples.shape[1]):
        f *= chk_factor_np(r, tuples[:, r])
    return int(np.sum(f, dtype=U64))


# ---------------------------------------------------------------- join-tree DP

def _group_sum(keys: np.ndarray, vals: List[np.ndarray]):
    """Distinct sorted keys and the (wrapping uint64) sum of each value array per key."""
    if keys.shape[0] == 0:
        return keys.astype(np.int64), [np.zeros(0, dtype=U64) for _ in vals]
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    starts = np.concatenate([[0], np.nonzero(ks[1:] != ks[:-1])[0] + 1])
    return ks[starts].astype(np.int64), [np.add.reduceat(v[order], starts, dtype=U64) for v in vals]


def _lookup(ukeys: np.ndarray, sums: np.ndarray, q: np.ndarray) -> np.ndarray:
    if ukeys.shape[0] == 0:
        return np.zeros(q.shape[0], dtype=U64)
    i = np.searchsorted(ukeys, q.astype(np.int64))
    i = np.minimum(i, ukeys.shape[0] - 1)
    hit = ukeys[i] == q
    return np.where(hit, sums[i], U64(0))


def join_tree_dp(query, root: Optional[int] = None, sels: Optional[List[np.ndarray]] = None):
    """(count, checksum) of an acyclic join by the sum-product recursion over its tree.

    Leaves up: a row's weight is the product over its children c of the summed
    weights of c's rows that match it; the checksum weight multiplies in the row's
    own factor mix64((rel << 32) | rid) | 1. ``sels`` optionally restricts each
    relation to the given rows (default: the predicate's eligible rows).
    """
    root = query.root if root is None else root
    n = len(query.rels)
    t = JoinTree(n, query.edges, root)
    if t.closing:
        raise ValueError("join-tree DP needs an acyclic join graph")
    if sels is None:
        sels = [eligible(r) for r in query.rels]
    agg = {}
    for j in t.postorder:
        rel = query.rels[j]
        sel = sels[j]
        cnt = np.ones(sel.shape[0], dtype=U64)
        val = chk_factor_np(j, sel)
        for c in t.children[j]:
            keys = rel.cols[t.pcol[c]][sel]
            uk, (ws, vs) = agg[c]
            cnt *= _lookup(uk, ws, keys)
            val *= _lookup(uk, vs, keys)
        if j == root:
            return int(np.sum(cnt, dtype=U64)), int(np.sum(val, dtype=U64))
        uk, sums = _group_sum(rel.cols[t.mycol[j]][sel], [cnt, val])
        agg[j] = (uk, sums)
    raise AssertionError("unreachable")


# ---------------------------------------------------------------- pruning phase

class _BloomFactory:
    def __init__(self, bits_per_key, k, block_bits, seed):
        self.bpk, self.k, self.B = bits_per_key, k, block_bits
        self.seed32 = filter_seed(seed)

    def build(self, keys, rows):
        # sized for the keys it receives: ceil(bits_per_key * |rows| / B) blocks
        nb = bf_nblocks(rows.shape[0], self.bpk, self.B)
        return (bf_build(keys, rows, nb, self.k, self.B, self.seed32), nb)

    def probe(self, f, keys, rows):
        words, nb = f
        return bf_probe(words, keys, rows, nb, self.k, self.B, self.seed32)


class _ExactFactory:
    """Exact key sets in place of filters (for the full-reducer pins)."""

    def build(self, keys, rows):
        return np.unique(keys[rows].astype(np.int64))

    def probe(self, f, keys, rows):
        return np.isin(keys[rows].astype(np.int64), f)


def sieve(query, bits_per_key: int = 8, k: int = 6, block_bits: int = 512, passes: int = 2,
          seed: int = 0, root: Optional[int] = None, exact: bool = False):
    """Survivor row ids of every relation after the pruning phase, and the filters.

    Returns ``(survivors, filters)``: survivors[r] is an ascending uint32 array;
    filters maps ('bwd', j) / ('fwd', j) / ('close', e) to (words, nblocks) -- or to
    a key set when ``exact``. A filter is sized for the rows it receives: Bloomjoin
    (Section 2.1 step 2) sizes the filter per tuple of the relation whose keys it
    holds, so a filter holding n survivors' keys gets ceil(bits_per_key * n / B)
    blocks.
    """
    root = query.root if root is None else root
    rels = query.rels
    t = JoinTree(len(rels), query.edges, root)
    fac = _ExactFactory() if exact else _BloomFactory(bits_per_key, k, block_bits, seed)
    elig = [eligible(r) for r in rels]
    S: Dict[int, np.ndarray] = {}
    F: Dict[tuple, object] = {}

    # backward pass: right-most relations first, each sieved by its children's filters
    for j in t.postorder:
        rows = elig[j]
        for c in t.children[j]:
            rows = rows[fac.probe(F[("bwd", c)], rels[j].cols[t.pcol[c]], rows)]
        S[j] = rows
        if j != root:
            F[("bwd", j)] = fac.build(rels[j].cols[t.mycol[j]], rows)

    if passes == 1:
        # closing edges: filter on the earlier end's survivors sieves the later end
        for e, (u, cu, v, cv) in enumerate(t.closing):
            F[("close", e)] = fac.build(rels[u].cols[cu], S[u])
            S[v] = S[v][fac.probe(F[("close", e)], rels[v].cols[cv], S[v])]
    elif passes == 2:
        # forward pass: root to leaves, each relation sieved by its parent's survivors
        for x in t.preorder:
            if x != root:
                rows = S[x]
                rows = rows[fac.probe(F[("fwd", x)], rels[x].cols[t.mycol[x]], rows)]
                for e, (u, cu, v, cv) in enumerate(t.closing):
                    if v == x:
                        rows = rows[fac.probe(F[("close", e)], rels[x].cols[cv], rows)]
                S[x] = rows
            for c in t.children[x]:
                F[("fwd", c)] = fac.build(rels[x].cols[t.pcol[c]], S[x])
            for e, (u, cu, v, cv) in enumerate(t.closing):
                if u == x:
                    F[("close", e)] = fac.build(rels[x].cols[cu], S[x])
    else:
        raise ValueError("passes must be 1 or 2")
    return [S[r] for r in range(len(rels))], F
