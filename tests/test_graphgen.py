"""The seeded input generators (no GPU): determinism, shapes and the two hash paths."""
import numpy as np
import torch

import graphgen


def test_cpu_and_device_hash_paths_agree():
    idx = torch.arange(0, 200000, dtype=torch.int64) * 7919 + 11
    for seed, stream in [(0, 0), (1, 5), (2**40 + 3, 1000)]:
        assert torch.equal(graphgen.mix_u32(idx, seed, stream),
                           graphgen.mix_u32_device_path(idx, seed, stream))


def test_rmat_deterministic_and_in_range():
    s1, d1, n = graphgen.rmat(12, 16, 3)
    s2, d2, _ = graphgen.rmat(12, 16, 3)
    assert n == 4096 and s1.numel() == 16 * 4096 and s1.dtype == torch.int32
    assert torch.equal(s1, s2) and torch.equal(d1, d2)
    assert int(s1.min()) >= 0 and int(s1.max()) < n and int(d1.max()) < n
    s3, _, _ = graphgen.rmat(12, 16, 4)
    assert not torch.equal(s1, s3)


def test_rmat_quadrant_skew():
    """Without the permutation, the top bit of src is set with probability c + d = 0.24."""
    s, d, n = graphgen.rmat(10, 64, 1, permute=False)
    top_src = (s.numpy() >> 9) & 1
    top_dst = (d.numpy() >> 9) & 1
    assert abs(top_src.mean() - 0.24) < 0.01
    assert abs(top_dst.mean() - 0.24) < 0.01  # b + d


def test_erdos_renyi_exact_m_simple():
    s, d, n = graphgen.erdos_renyi(1024, 8192, 0)
    s, d = s.numpy().astype(np.int64), d.numpy().astype(np.int64)
    assert s.size == 8192 and np.all(s != d)
    keys = np.minimum(s, d) * n + np.maximum(s, d)
    assert np.unique(keys).size == 8192
    s2, _, _ = graphgen.erdos_renyi(1024, 8192, 0)
    assert np.array_equal(s, s2.numpy())


def test_erdos_renyi_dense_limit():
    s, d, n = graphgen.erdos_renyi(12, 66, 2)
    assert s.numel() == 66


def test_rmat_unique_target_and_range():
    s, d, n = graphgen.rmat_unique(3000, 20000, 9)
    s, d = s.numpy().astype(np.int64), d.numpy().astype(np.int64)
    assert n == 3000 and s.max() < n and d.max() < n and np.all(s != d)
    keys = np.minimum(s, d) * n + np.maximum(s, d)
    assert np.unique(keys).size == s.size
    assert s.size == 20000


def test_batch_spec():
    spec = graphgen.batch_suite_spec(64, seed=4)
    assert len(spec) == 64
    assert all(256 <= g.n <= 65536 for g in spec)
    assert all(4 <= g.avg_degree <= 64 for g in spec)
    assert [g.kind for g in spec[:4]] == ["er", "rmat", "er", "rmat"]
    assert spec == graphgen.batch_suite_spec(64, seed=4)


def test_poisson_arrivals():
    t = graphgen.poisson_arrivals(20000, qps=100.0, seed=5)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 20000 - 0.01) < 0.0005


def test_vertex_labels_in_range_and_seeded():
    a = graphgen.vertex_labels(5000, 4, 3)
    assert a.dtype == torch.int32 and int(a.min()) >= 0 and int(a.max()) < 4
    assert torch.equal(a, graphgen.vertex_labels(5000, 4, 3))
    assert not torch.equal(a, graphgen.vertex_labels(5000, 4, 4))
    counts = torch.bincount(a.long(), minlength=4)
    assert int(counts.min()) > 1000  # roughly uniform
