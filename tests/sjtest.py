"""Helpers shared by the GPU tests: upload a workload, run the plan, compare with the oracle."""
import numpy as np
import torch

import oracle
import paper_2308_16370_amd as sj

KIND_NAME = {sj.SJ_FILTER_BACKWARD: "bwd", sj.SJ_FILTER_FORWARD: "fwd", sj.SJ_FILTER_CLOSING: "close"}


def to_device(q, dev="cuda:0"):
    """sj.Rel list for a workloads.Query; columns shared between relations upload once."""
    cache = {}
    rels = []
    for r in q.rels:
        cols = []
        for c in r.cols:
            key = id(c)
            if key not in cache:
                cache[key] = torch.from_numpy(np.ascontiguousarray(c, dtype=np.int32)).to(dev)
            cols.append(cache[key])
        rels.append(sj.Rel(cols, r.pred))
    return rels


def make_plan(q, ctx=None, **opts):
    ctx = ctx or sj.Context(0)
    return sj.Plan(ctx, to_device(q), q.edges, root=q.root, **opts)


def lexsort_rows(t):
    if t.shape[0] == 0:
        return t
    return t[np.lexsort(tuple(t[:, i] for i in reversed(range(t.shape[1]))))]


def preorder(q):
    return oracle.JoinTree(len(q.rels), q.edges, q.root).preorder


def check_sorted_in_preorder(q, t):
    """Tuples are strictly increasing when compared in the plan's preorder of relations."""
    if t.shape[0] < 2:
        return
    cols = t[:, preorder(q)].astype(np.int64)
    d = np.diff(cols, axis=0)
    nz = d != 0
    assert nz.any(axis=1).all(), "duplicate tuple"
    first = np.argmax(nz, axis=1)
    assert (d[np.arange(d.shape[0]), first] > 0).all(), "not sorted"


def check_sieve(q, plan, bits_per_key, k, block_bits, passes, seed):
    """Filter words and survivor lists equal the oracle's, bit for bit."""
    S, F = oracle.sieve(q, bits_per_key=bits_per_key, k=k, block_bits=block_bits, passes=passes,
                        seed=seed, root=q.root)
    for i in range(len(q.rels)):
        got = plan.survivors(i).cpu().numpy().astype(np.uint32)
        assert np.array_equal(got, S[i]), "survivors of relation %d differ" % i
    nf = plan.filter_count()
    assert nf == len(F)
    for f in range(nf):
        d = plan.filter_desc(f)
        words, nb = F[(KIND_NAME[d["kind"]], d["index"])]
        assert d["nblocks"] == nb
        got = plan.filter_words(f).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, words), "filter %r differs" % (d,)
    return S, F
