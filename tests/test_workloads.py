"""The input generators: the torch path of the power-law edge generator (used to
generate the full-size triangle workload quickly on the GPU) draws exactly the edges
of the numpy path, including when duplicates force several rounds of draws."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("nedges,nverts,gamma,seed", [
    (1000, 64, 2.1, 1),        # dense: many duplicates, several rounds of draws
    (5000, 120, 1.8, 2),
    (20000, 4096, 2.1, 0x5EED0004),
    (1, 8, 2.1, 3),
])
def test_torch_edges_equal_numpy_edges(nedges, nverts, gamma, seed):
    s0, d0 = W.powerlaw_edges(nedges, nverts, gamma, seed)
    s1, d1 = W.powerlaw_edges(nedges, nverts, gamma, seed, device="cpu")
    assert s1.dtype == s0.dtype == np.int32
    assert np.array_equal(s0, s1) and np.array_equal(d0, d1)
    key = s0.astype(np.int64) * nverts + d0
    assert np.unique(key).shape[0] == nedges and not np.any(s0 == d0)


def test_config4_device_path_equals_numpy_path():
    a = W.config4(scale=1 / 256)
    b = W.config4(scale=1 / 256, device="cpu")
    for x, y in zip(a.rels[0].cols, b.rels[0].cols):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("index", range(10))
def test_serving_query_gpu_path_equals_cpu_path(index):
    """The serving mix's device path (run here on the CPU device) draws exactly the
    columns of its numpy path, for chains and stars, skewed and uniform keys."""
    from workloads import serving as S
    sp = S.draw_spec(0x5EED0005, index, 0, min_rows=1000, max_rows=30_000)
    if index == 0:
        sp = S.QuerySpec(sp.index, 0, sp.kind, sp.rows, 0.0, sp.seed)   # uniform keys
    q = S.query_cpu(sp)
    rels, edges = S.query_gpu(sp, device="cpu")
    assert edges == q.edges
    for rel, (cols, pred) in zip(q.rels, rels):
        assert pred == rel.pred
        for a, b in zip(rel.cols, cols):
            assert np.array_equal(a, b.numpy())
