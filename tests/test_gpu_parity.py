"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Filter words, survivor lists, result count, checksum and every result tuple are
compared exactly (all of the path is integer arithmetic).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_16370_amd as sj
import workloads as W
from sjtest import check_sieve, check_sorted_in_preorder, lexsort_rows, make_plan

pytestmark = pytest.mark.gpu


def run_and_compare(q, bits_per_key=8, k=6, block_bits=512, passes=2, seed=7, sieve=True, **opts):
    plan = make_plan(q, bits_per_key=bits_per_key, k=k, block_bits=block_bits, passes=passes, seed=seed, **opts)
    plan.build_filters()
    plan.sieve()
    if sieve:
        check_sieve(q, plan, bits_per_key, k, block_bits, passes, seed)
    cnt, chk = plan.join()
    tup = plan.result().cpu().numpy().astype(np.uint32)
    ref, rcnt, rchk = oracle.hash_join(q)
    assert (cnt, chk) == (rcnt, rchk)
    assert tup.shape == (rcnt, len(q.rels))
    # 3-cycles are written by the intersection walk (walk order); other plans decode the
    # tree in preorder (sorted)
    if not (len(q.rels) == 3 and len(q.edges) >= 3):
        check_sorted_in_preorder(q, tup)
    assert np.array_equal(lexsort_rows(tup), ref)
    return plan, tup


ACYCLIC = ["chain", "star", "tree", "pair"]


@pytest.mark.parametrize("seed", range(120))
def test_tiny_random_acyclic(seed):
    q = W.tiny_random(7000 + seed, kind=ACYCLIC[seed % 4])
    run_and_compare(q, bits_per_key=[2, 4, 8][seed % 3], k=[1, 3, 6][seed % 3],
                    block_bits=[256, 512, 1024][(seed // 3) % 3], passes=1 + seed % 2, seed=seed)


@pytest.mark.parametrize("seed", range(60))
def test_tiny_random_cyclic(seed):
    q = W.tiny_random(8000 + seed, kind=["triangle", "cycle4", "selfjoin"][seed % 3])
    passes = 1 + seed % 2
    plan = make_plan(q, bits_per_key=4, k=3, passes=passes, seed=seed)
    plan.build_filters()
    plan.sieve()
    check_sieve(q, plan, 4, 3, 512, passes, seed)
    cnt, chk = plan.join()
    ref, rcnt, rchk = oracle.hash_join(q)
    assert (cnt, chk) == (rcnt, rchk)
    tup = plan.result().cpu().numpy().astype(np.uint32)
    assert np.array_equal(lexsort_rows(tup), ref)


def test_triangle_small():
    q = W.triangle(6000, 1500, 2.1, seed=9)
    plan, tup = run_and_compare(q, seed=4)
    assert tup.shape[0] > 1000 and tup.shape[0] % 3 == 0


def test_psyn_with_redundant_closing_edge():
    q = W.psyn(20000, 100, 3, seed=6)
    q.edges.append((0, 0, 2, 0))      # R.x = T.x is implied; it becomes a closing edge
    plan, tup = run_and_compare(q, seed=2)
    assert tup.shape[0] == 100 * 27


def test_config1_full_scale():
    q = W.config1()
    plan, tup = run_and_compare(q, bits_per_key=10, k=7, seed=0x5EED0001)
    assert 200_000 < tup.shape[0] < 800_000


@pytest.mark.parametrize("passes", [1, 2])
def test_config2_reduced(passes):
    q = W.config2(scale=0.01)
    run_and_compare(q, bits_per_key=8, k=6, passes=passes, seed=3)


@pytest.mark.parametrize("k", [2, 4, 6])
def test_exact_k_instances(k):
    """The probe and build kernels have instances for k = 2, 4 and 6 with k fixed at
    compile time (other k use a general instance); every filter word, survivor and tuple
    against the oracle at 100K rows per relation (many tiles per scan)."""
    q = W.config2(scale=0.01)
    run_and_compare(q, bits_per_key=8, k=k, seed=9)


@pytest.mark.parametrize("two_launches", [False, True])
@pytest.mark.parametrize("grid", [64, 256, 1024])
def test_sieve_scan_launch_forms(two_launches, grid):
    """A sieve step that writes a survivor list runs as one launch (each workgroup takes a
    ticket and finds its output offset by a look-back over the workgroups before it) or,
    with SJ_FLAG_SIEVE_TWO_LAUNCHES, as a probe and a compaction launch; both against the
    oracle's survivors and tuples, over grids of 64 to 1024 workgroups (1024 workgroups
    do not all fit on the device at once) and ragged row counts."""
    q = W.config2(scale=0.013)
    run_and_compare(q, bits_per_key=8, k=6, seed=11, probe_grid=grid,
                    flags=sj.SJ_FLAG_SIEVE_TWO_LAUNCHES if two_launches else 0)


@pytest.mark.parametrize("n1", [(1 << 20) - 1, 1 << 20, (1 << 20) + 1])
def test_bucket_sort_tile_boundary(n1):
    """The radix sort of a bucketed relation takes 512-entry tiles up to 2^20 entries and
    2048-entry tiles above, chosen on the device from the sieved count. R0 holds every key
    of a 2^19-key domain once, so every row of R1 survives and R1's bucketed list is
    exactly n1 entries: filters, survivors, count, checksum and tuples against the oracle
    on both sides of the switch."""
    rng = np.random.default_rng(n1)
    d = 1 << 19
    r0 = W.Relation("R0", [rng.permutation(d).astype(np.int32)])
    r1 = W.Relation("R1", [rng.integers(0, d, n1).astype(np.int32)])
    q = W.Query("tile_boundary", [r0, r1], [(0, 0, 1, 0)], 0)
    plan, tup = run_and_compare(q, seed=3)
    assert tup.shape[0] == n1


def test_star_reduced():
    q = W.config3(scale=0.01)
    plan, tup = run_and_compare(q, bits_per_key=8, k=6, seed=5)


def test_psyn():
    q = W.psyn(20000, 100, 5, seed=2)
    plan, tup = run_and_compare(q, seed=9)
    assert tup.shape[0] == 100 * 5 ** 3


def test_single_relation_and_empty():
    x = np.arange(-5, 20, dtype=np.int32)
    q = W.Query("one", [W.Relation("R", [x], pred=(0, 0, 10))], [])
    run_and_compare(q)
    e = np.zeros(0, dtype=np.int32)
    q = W.Query("empty", [W.Relation("R", [x]), W.Relation("S", [e])], [(0, 0, 1, 0)])
    run_and_compare(q)
    q = W.Query("none", [W.Relation("R", [x], pred=(0, 100, 200)), W.Relation("S", [x.copy()])], [(0, 0, 1, 0)])
    run_and_compare(q)


def test_capacity_and_state_errors():
    q = W.config1(scale=0.02)
    plan = make_plan(q, bits_per_key=10, k=7)
    with pytest.raises(sj.SjError) as e:
        plan.sieve()
    assert e.value.code == sj.SJ_ERR_STATE
    plan.build_filters()
    plan.sieve()
    cnt, chk = plan.join()
    assert cnt > 1
    small = torch.empty((cnt - 1, 3), dtype=torch.int32, device="cuda:0")
    with pytest.raises(sj.SjError) as e:
        plan.result(small)
    assert e.value.code == sj.SJ_ERR_CAPACITY
    # re-running every phase on the same plan gives the same result
    t1 = plan.result().cpu()
    plan.build_filters()
    plan.sieve()
    assert plan.join() == (cnt, chk)
    assert torch.equal(plan.result().cpu(), t1)
