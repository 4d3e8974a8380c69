"""GPU parity of the segmented-intersection operator (tc_segmented_intersect: a merge-path
intersection of N+(u) and N+(v) for every DAG edge) and of the diamond query
(tc_count_diamonds) against the oracle.

Counts and supports are integers and the DAG is bit-exact with the oracle's, so the bar is
equality: the total, every edge's support, and the number of diamonds.
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


def _pipe(tc, n, s, d, *, order=0, offset_bytes=4):
    p = tc.Pipeline(n, max(len(s), 1), offset_bytes=offset_bytes, order=order)
    p.build(_dev(s), _dev(d))
    p.orient()
    return p


def _oracle_support(n, s, d, order=0):
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    return oracle.edge_support(dp, dc)


def _check(tc, n, s, d, order=0, offset_bytes=4, diamonds=True):
    p = _pipe(tc, n, s, d, order=order, offset_bytes=offset_bytes)
    T, want = _oracle_support(n, s, d, order)
    p.intersect()
    assert p.intersect_total() == T
    p.intersect(support=True)
    assert p.intersect_total() == T
    np.testing.assert_array_equal(p.supports().cpu().numpy().view(np.uint32), want)
    if diamonds:
        p.diamonds()
        assert p.diamond_count() == oracle.diamonds(n, np.asarray(s), np.asarray(d))
    return p


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_intersect_golden_fixtures(tc, fx):
    _say("intersect golden", fx.name)
    for order in (0, 1):
        for ob in (4, 8):
            _check(tc, fx.n, fx.src, fx.dst, order, ob)


def test_intersect_closed_forms(tc):
    # K_n: C(n,3) triangles, every edge in n-2 of them, C(n,2) * C(n-2,2) diamonds
    for n in (3, 4, 9, 40):
        n_, s, d = pins.complete(n)
        p = _check(tc, n_, s, d)
        assert p.intersect_total() == n * (n - 1) * (n - 2) // 6
        assert p.diamond_count() == (n * (n - 1) // 2) * ((n - 2) * (n - 3) // 2)
    # wheel W_k (k rim vertices, k >= 4): k triangles; each spoke lies in 2, each rim
    # edge in 1, so the k spokes give k diamonds
    for k in (4, 7, 30):
        s = [0] * k + list(range(1, k + 1))
        d = list(range(1, k + 1)) + [i % k + 1 for i in range(1, k + 1)]
        p = _check(tc, k + 1, s, d)
        assert p.intersect_total() == k
        assert p.diamond_count() == k


def test_intersect_random_tiny(tc):
    for seed in range(40):
        rng = np.random.default_rng(1300 + seed)
        n = int(rng.integers(1, 48))
        n, s, d = pins.random_simple(n, float(rng.choice([0.1, 0.3, 0.6, 1.0])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        _say("intersect tiny seed", seed, "n", n)
        for order in (0, 1):
            _check(tc, n, s, d, order, 4 + 4 * (seed % 2))


@pytest.mark.parametrize("scale,seed", [(10, 1), (14, 2), (16, 3)])
def test_intersect_rmat(tc, scale, seed):
    s, d, n = graphgen.rmat(scale, 16, seed)
    _say("intersect rmat", scale)
    for order in (0, 1):
        _check(tc, n, s.numpy(), d.numpy(), order, diamonds=order == 0)


def test_intersect_config1_and_hub(tc):
    for seed in range(3):
        s, d, n = graphgen.erdos_renyi(1024, 8192, seed)
        _check(tc, n, s.numpy(), d.numpy())
    # a hub adjacent to everything: long stretches under id order
    rng = np.random.default_rng(12)
    n = 4001
    s = np.concatenate([np.zeros(4000, dtype=np.int64), rng.integers(1, n, 30000)])
    d = np.concatenate([np.arange(1, n), rng.integers(1, n, 30000)])
    for order in (0, 1):
        _check(tc, n, s, d, order)


def test_intersect_capacity_and_degenerate(tc):
    from paper_1909_02127_amd import _lib
    n, s, d = pins.complete(8)  # 28 edges
    p = _pipe(tc, n, s, d)
    # a column capacity below m is reported on the device
    ws = torch.empty(_lib.tc_segmented_intersect_workspace(n, 27), dtype=torch.uint8,
                     device="cuda")
    m_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    total = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    _lib.tc_segmented_intersect(n, p.dag_ptr, p.dag_col[:27], total, m_out, ws)
    torch.cuda.synchronize()
    assert int(m_out.item()) == -_lib.TC_ERR_CAPACITY
    assert int(total.item()) == 0
    for n, s, d in [(0, [], []), (1, [], []), (6, [0, 1, 2], [1, 2, 3]), (5, [2, 2], [2, 2]),
                    (3, [0, 1, 0], [1, 2, 2])]:
        _check(tc, n, s, d)


def test_intersect_rmat_scale20_full(tc):
    """The benchmark graph: the total, every edge's support and the diamonds against the
    oracle."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    p = tc.Pipeline(n, s.numel(), offset_bytes=4)
    p.build(s, d)
    p.orient()
    p.intersect(support=True)
    T = p.intersect_total()
    sup = p.supports().cpu().numpy().view(np.uint32)
    p.diamonds()
    dia = p.diamond_count()
    _say("scale 20 intersect: oracle")
    hs, hd = s.cpu().numpy(), d.cpu().numpy()
    T0, want = _oracle_support(n, hs, hd)
    assert T == T0
    np.testing.assert_array_equal(sup, want)
    # diamonds: the sum over edges of C(s, 2) of the oracle's supports (an identity the
    # oracle's own pins check against its diamond enumeration)
    w = want.astype(np.uint64)
    assert dia == int((w * (w - 1) // 2).sum())


def test_intersect_wide_column_offsets(tc):
    """An edge capacity of 2^30 or more makes the merge kernel address the column array with
    64-bit offsets (below it, 32-bit offsets from the array's base); same counts."""
    from paper_1909_02127_amd import _lib
    s, d, n = graphgen.rmat(10, 16, 4)
    p = _pipe(tc, n, s.numpy(), d.numpy())
    T, want = _oracle_support(n, s.numpy(), d.numpy())
    cap = (1 << 30) + 1
    col = torch.zeros(cap, dtype=torch.int32, device="cuda")
    m = p.dag_col.numel()
    col[:m].copy_(p.dag_col)
    sup = torch.full((cap,), 7, dtype=torch.int32, device="cuda")
    ws = torch.empty(_lib.tc_segmented_intersect_workspace(n, cap), dtype=torch.uint8,
                     device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    m_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.tc_segmented_intersect(n, p.dag_ptr, col, total, m_out, ws, support=sup)
    torch.cuda.synchronize()
    mm = int(m_out.item())
    assert mm == int(p.dag_ptr[-1].item()) and int(total.item()) == T
    np.testing.assert_array_equal(sup[:mm].cpu().numpy().view(np.uint32), want)
    _lib.tc_segmented_intersect(n, p.dag_ptr, col, total, m_out, ws)
    torch.cuda.synchronize()
    assert int(total.item()) == T
