"""Inserts into built filters (Section 2.4): a tuple added to a relation changes the
relation's filter only when the filter does not yet contain its key, and those keys
are the ones to propagate to adjacent relations.

Parity: for every filter of a plan (backward, forward, closing), inserting a batch of
keys leaves exactly the oracle's words (the old words with every key's pattern set),
reports exactly the keys the old filter contained, and counts the others; a probe
afterwards finds every key. Propagation: new rows appended to a chain's leaf are
inserted into the leaf's filter; the parent rows whose key matches a newly inserted
key go into the parent's filter, and so on. The maintained filters then contain every
key that truly joins in the grown query.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import to_device

pytestmark = pytest.mark.gpu

OPTS = dict(bits_per_key=8, k=6, block_bits=512, passes=2, seed=31)


def built_plan(q, **kw):
    plan = sj.Plan(sj.Context(0), to_device(q), q.edges, root=q.root, **dict(OPTS, **kw))
    plan.build_filters()
    plan.sieve()
    return plan


@pytest.mark.parametrize("kind", ["chain", "triangle"])
def test_insert_and_probe_parity(kind):
    q = W.chain(4, 3000, 2000, 0.6, 0x5EED00D1) if kind == "chain" else W.triangle(8000, 900, 2.1, 0x5EED00D2)
    plan = built_plan(q)
    seed32 = oracle.filter_seed(OPTS["seed"])
    rng = np.random.default_rng(5)
    kinds = set()
    for f in range(plan.filter_count()):
        d = plan.filter_desc(f)
        kinds.add(d["kind"])
        words = plan.filter_words(f).cpu().numpy().view(np.uint32).copy()
        src = q.rels[d["src_rel"]].cols[d["src_col"]]
        keys = np.concatenate([rng.choice(src, 200),                                  # mostly present
                               rng.integers(-2**31, 2**31, 300, dtype=np.int64).astype(np.int32),
                               np.array([-2**31, 2**31 - 1, -1, 0, 0, 0], dtype=np.int32)])
        want_words, want_flags = oracle.bf_insert(words, keys, d["nblocks"], OPTS["k"], OPTS["block_bits"], seed32)
        kd = torch.from_numpy(keys).cuda()
        pflags, missing = plan.filter_probe(f, kd)
        assert np.array_equal(pflags.cpu().numpy(), want_flags) and missing == int((~want_flags).sum())
        flags, inserted = plan.filter_insert(f, kd)
        assert np.array_equal(flags.cpu().numpy(), want_flags)
        assert inserted == int((~want_flags).sum()) and inserted > 0
        assert plan.filter_desc(f)["nblocks"] == d["nblocks"]
        assert np.array_equal(plan.filter_words(f).cpu().numpy().view(np.uint32), want_words)
        after, missing = plan.filter_probe(f, kd)
        assert bool(after.all()) and missing == 0
    assert sj.SJ_FILTER_BACKWARD in kinds and sj.SJ_FILTER_FORWARD in kinds
    if kind == "triangle":
        assert sj.SJ_FILTER_CLOSING in kinds
    empty, n = plan.filter_insert(0, torch.empty(0, dtype=torch.int32, device="cuda:0"))
    assert n == 0 and empty.numel() == 0


def test_state_and_sharing_errors():
    q = W.chain(3, 500, 300, 0.0, 0x5EED00D3)
    plan = sj.Plan(sj.Context(0), to_device(q), q.edges, **OPTS)
    keys = torch.arange(10, dtype=torch.int32, device="cuda:0")
    with pytest.raises(sj.SjError) as e:        # nothing built yet
        plan.filter_probe(0, keys)
    assert e.value.code == sj.SJ_ERR_STATE
    with pytest.raises(sj.SjError) as e:
        plan.filter_insert(99, keys)
    assert e.value.code == sj.SJ_ERR_INVALID
    cache = sj.FilterCache(8 << 20)
    shared = sj.Plan(sj.Context(0), to_device(q), q.edges, filter_cache=cache, **OPTS)
    shared.build_filters()
    bwd = [f for f in range(shared.filter_count()) if shared.filter_cached(f)]
    assert bwd
    shared.filter_probe(bwd[0], keys)           # probing a shared filter is fine
    with pytest.raises(sj.SjError) as e:
        shared.filter_insert(bwd[0], keys)
    assert e.value.code == sj.SJ_ERR_STATE


def test_propagating_appended_rows_along_a_chain():
    """R1 - R2 - R3 rooted at R1; 600 new rows appended to R3. Their keys go into R3's
    backward filter; R2 rows matching a newly inserted key put theirs into R2's
    backward filter. Every key of the grown query that truly joins is then contained."""
    q = W.chain(3, 4000, 6000, 0.4, 0x5EED00D4)
    plan = built_plan(q)
    fb = {plan.filter_desc(f)["index"]: f for f in range(plan.filter_count())
          if plan.filter_desc(f, nblocks=False)["kind"] == sj.SJ_FILTER_BACKWARD}
    rng = np.random.default_rng(9)
    new_r3 = [rng.integers(0, 9000, 600).astype(np.int32) for _ in range(2)]
    # R3 (leaf): its backward filter holds its parent-edge key, column 0
    k3 = torch.from_numpy(new_r3[0]).cuda()
    flags3, n3 = plan.filter_insert(fb[2], k3)
    missing3 = k3[~flags3]
    # R2 rows whose child-edge key (column 1) matches a newly inserted key can now pass
    r2c0, r2c1 = (torch.from_numpy(c).cuda() for c in q.rels[1].cols)
    newly = torch.isin(r2c1, missing3)
    flags2, n2 = plan.filter_insert(fb[1], r2c0[newly].contiguous())
    assert n3 > 0
    # the grown query: keys that truly join must be contained
    g3 = [np.concatenate([q.rels[2].cols[c], new_r3[c]]) for c in range(2)]
    must3 = torch.from_numpy(np.unique(g3[0])).cuda()
    ok3, miss3 = plan.filter_probe(fb[2], must3)
    assert miss3 == 0
    joins2 = np.isin(q.rels[1].cols[1], g3[0])           # R2 rows with a partner in the grown R3
    must2 = torch.from_numpy(np.unique(q.rels[1].cols[0][joins2])).cuda()
    ok2, miss2 = plan.filter_probe(fb[1], must2)
    assert miss2 == 0


def revived_chain(seed):
    """A 4-chain whose leaf holds only keys below 50 on its joining column, so the parent
    rows with keys 50..99 dangle until new leaf rows bring those keys (propagation then
    climbs several levels)."""
    q = W.chain(4, [1500, 1200, 900, 600], 100, 0.0, seed)
    q.rels[3].cols[0] = (q.rels[3].cols[0] % 50).astype(np.int32)
    return q


@pytest.mark.parametrize("seed", range(4))
def test_propagate_parity(seed):
    """sj_filter_propagate leaves exactly the oracle's backward filters (oracle.propagate)
    and reports the same counts of keys each filter did not hold."""
    q = revived_chain(0x5EED0D10 + seed) if seed < 2 else W.star(3000, 3, 400, 0.5, 0x5EED0D10 + seed)
    rel = 3 if seed < 2 else 1 + seed % 3
    plan = built_plan(q, passes=1)
    seed32 = oracle.filter_seed(OPTS["seed"])
    _, F = oracle.sieve(q, bits_per_key=8, k=6, block_bits=512, passes=1, seed=OPTS["seed"], root=q.root)
    bwd = {j: F[("bwd", j)] for (kind, j) in F if kind == "bwd"}
    rng = np.random.default_rng(seed)
    nnew = 200
    if seed < 2:
        new_cols = [rng.integers(50, 100, size=nnew).astype(np.int32), rng.integers(0, 100, size=nnew).astype(np.int32)]
    else:
        dim = q.rels[rel]
        new_cols = [rng.integers(400, 500, size=nnew).astype(np.int32), rng.integers(0, 400, size=nnew).astype(np.int32)]
    F2, want = oracle.propagate(q, bwd, rel, new_cols, 6, 512, seed32)
    got = plan.propagate(rel, [torch.from_numpy(c).to("cuda:0") for c in new_cols])
    assert got == want
    if seed < 2:
        assert sum(1 for x in want if x) >= 2, want   # several levels
    for f in range(plan.filter_count()):
        d = plan.filter_desc(f)
        if d["kind"] != sj.SJ_FILTER_BACKWARD:
            continue
        words, nb = F2[d["index"]]
        assert d["nblocks"] == nb
        assert np.array_equal(plan.filter_words(f).cpu().numpy().view(np.uint32), words), d


def gpu_counters(cf, nb, B=512):
    """uint8 [nblocks, B] from the counter words (nibble p % 8 of word b * B / 8 + p / 8)."""
    w = cf.counters().cpu().numpy().view(np.uint32).reshape(nb, B // 8)
    out = np.empty((nb, B), dtype=np.uint8)
    for t in range(8):
        out[:, t::8] = (w >> (4 * t)) & 15
    return out


@pytest.mark.parametrize("kind", ["chain", "star"])
def test_counting_filter_parity(kind):
    """The counting twin of every backward filter: its support is the plan's filter,
    its counters equal the oracle's for the keys the filter was built from, and after
    deleting a third of those keys and inserting others the counters, the exported
    filter and the plan's filter after apply() equal the oracle's."""
    q = W.chain(3, [4000, 3000, 2500], 3000, 0.3, 0x5EED0D20) if kind == "chain" else \
        W.star(6000, 3, 800, 0.4, 0x5EED0D21)
    plan = built_plan(q, passes=1)
    seed32 = oracle.filter_seed(OPTS["seed"])
    _, F = oracle.sieve(q, bits_per_key=8, k=6, block_bits=512, passes=1, seed=OPTS["seed"], root=q.root)
    t = oracle.JoinTree(len(q.rels), q.edges, q.root)
    rng = np.random.default_rng(1)
    for f in range(plan.filter_count()):
        d = plan.filter_desc(f)
        if d["kind"] != sj.SJ_FILTER_BACKWARD:
            continue
        j, nb = d["index"], d["nblocks"]
        # the keys the build inserted: rows of j passing its predicate and children's filters
        R = q.rels[j]
        ok = np.ones(R.nrows, dtype=bool)
        if R.pred is not None:
            pc, lo, hi = R.pred
            ok &= (R.cols[pc] >= lo) & (R.cols[pc] < hi)
        for c in t.children[j]:
            w, nbc = F[("bwd", c)]
            ok &= oracle.bf_probe(w, R.cols[t.pcol[c]], None, nbc, 6, 512, seed32)
        keys = R.cols[t.mycol[j]][ok]
        cf = plan.counting_filter(f)
        want = oracle.cf_update(np.zeros((nb, 512), dtype=np.uint8), keys, +1, nb, 6, 512, seed32)
        assert np.array_equal(gpu_counters(cf, nb), want)
        assert np.array_equal(cf.export().cpu().numpy().view(np.uint32), plan.filter_words(f).cpu().numpy().view(np.uint32))
        gone = keys[rng.random(keys.shape[0]) < 0.33]
        extra = rng.integers(-2**31, 2**31, size=100).astype(np.int32)
        cf.delete(torch.from_numpy(gone).to("cuda:0"))
        cf.insert(torch.from_numpy(extra).to("cuda:0"))
        want = oracle.cf_update(oracle.cf_update(want, gone, -1, nb, 6, 512, seed32), extra, +1, nb, 6, 512, seed32)
        assert np.array_equal(gpu_counters(cf, nb), want)
        words = oracle.cf_export(want)
        assert np.array_equal(cf.export().cpu().numpy().view(np.uint32), words)
        flags, miss = cf.probe(torch.from_numpy(keys).to("cuda:0"))
        assert miss == int((~oracle.bf_probe(words, keys, None, nb, 6, 512, seed32)).sum())
        cf.apply()
        assert np.array_equal(plan.filter_words(f).cpu().numpy().view(np.uint32), words)
        del cf
