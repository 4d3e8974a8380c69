"""GPU parity of tc_edge_support (triangles on every oriented edge) against the oracle.

Supports are integers aligned with the DAG columns, and the DAG is bit-exact with
the oracle's, so the bar is element-by-element equality.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests import goldens, pins

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_02127_amd as tc
    return tc


def _dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.int32)).cuda()


def _gpu_support(tc, n, s, d, *, order=0, offset_bytes=4, tune=None):
    p = tc.Pipeline(n, max(len(s), 1), offset_bytes=offset_bytes, order=order, tune=tune)
    p.build(_dev(s), _dev(d))
    p.orient()
    p.edge_support()
    sup = p.supports().cpu().numpy().view(np.uint32)
    return p, sup


def _oracle_support(n, s, d, order=0):
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    return oracle.edge_support(dp, dc)


def _check(tc, n, s, d, order=0, offset_bytes=4, tune=None):
    p, sup = _gpu_support(tc, n, s, d, order=order, offset_bytes=offset_bytes, tune=tune)
    T, want = _oracle_support(n, s, d, order)
    np.testing.assert_array_equal(sup, want)
    assert int(p.total.item()) == T


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_support_golden_fixtures(tc, fx):
    _say("support golden", fx.name)
    for order in (0, 1):
        for ob in (4, 8):
            _check(tc, fx.n, fx.src, fx.dst, order, ob)


def test_support_random_tiny(tc):
    for seed in range(40):
        rng = np.random.default_rng(900 + seed)
        n = int(rng.integers(1, 48))
        n, s, d = pins.random_simple(n, float(rng.choice([0.1, 0.3, 0.6, 1.0])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        _say("support tiny seed", seed, "n", n)
        for order in (0, 1):
            _check(tc, n, s, d, order, 4 + 4 * (seed % 2))


@pytest.mark.parametrize("scale,seed", [(10, 1), (14, 2), (16, 3)])
def test_support_rmat(tc, scale, seed):
    s, d, n = graphgen.rmat(scale, 16, seed)
    _say("support rmat", scale)
    for order in (0, 1):
        _check(tc, n, s.numpy(), d.numpy(), order)


def test_support_config1_and_hub(tc):
    for seed in range(3):
        s, d, n = graphgen.erdos_renyi(1024, 8192, seed)
        _check(tc, n, s.numpy(), d.numpy())
    rng = np.random.default_rng(11)
    n = 4001
    s = np.concatenate([np.zeros(4000, dtype=np.int64), rng.integers(1, n, 30000)])
    d = np.concatenate([np.arange(1, n), rng.integers(1, n, 30000)])
    for order in (0, 1):
        _check(tc, n, s, d, order)
    n, s, d = pins.complete(150)
    _check(tc, n, s, d, 1)


def test_support_with_split_sources(tc):
    """Equal-work quanta (tc_tune.split_log2): every part of a split source adds its own
    edge counts; the supports must not change."""
    tune = {"split_log2": 3, "small_max": 16}
    s, d, n = graphgen.rmat(12, 16, 8)
    for order in (0, 1):
        _check(tc, n, s.numpy(), d.numpy(), order, tune=tune)
    n, s, d = pins.complete(60)
    _check(tc, n, s, d, 1, tune=tune)


@pytest.mark.parametrize("kicks", [-1, 1])
def test_support_probe_fallback_modes(tc, kicks):
    tune = {"max_kicks": kicks}
    s, d, n = graphgen.rmat(12, 16, 8)
    for order in (0, 1):
        _check(tc, n, s.numpy(), d.numpy(), order, tune=tune)
    n, s, d = pins.complete(60)
    _check(tc, n, s, d, 0, tune=tune)


def test_support_capacity_and_degenerate(tc):
    from paper_1909_02127_amd import _lib
    n, s, d = pins.complete(8)  # 28 edges
    p, sup = _gpu_support(tc, n, s, d)
    assert sup.size == 28 and np.all(sup == 6)
    small = torch.full((27,), -7, dtype=torch.int32, device="cuda")
    _lib.tc_edge_support(n, p.dag_ptr, p.dag_col, small, p.support_m, p.ws_support)
    torch.cuda.synchronize()
    assert int(p.support_m.item()) == -3
    assert bool((small == -7).all())
    for n, s, d in [(0, [], []), (1, [], []), (6, [0, 1, 2], [1, 2, 3]), (5, [2, 2], [2, 2])]:
        _, sup = _gpu_support(tc, n, s, d)
        assert not sup.any()


def test_support_rmat_scale20_full(tc):
    """The benchmark graph: every edge's support against the oracle."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    p = tc.Pipeline(n, s.numel(), offset_bytes=4)
    p.build(s, d)
    p.orient()
    p.edge_support()
    sup = p.supports().cpu().numpy().view(np.uint32)
    _say("scale 20 support: oracle")
    T, want = _oracle_support(n, s.cpu().numpy(), d.cpu().numpy())
    np.testing.assert_array_equal(sup, want)
    assert int(sup.sum(dtype=np.uint64)) == 3 * T
