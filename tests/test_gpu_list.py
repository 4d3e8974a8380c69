"""GPU parity of tc_list_triangles (the match set M) against the CPU oracle.

Under one orientation every triangle has exactly one row (u, v, w), so the rows
are unique; the GPU writes the rows of one source in no particular order, so
both listings are compared after a lexicographic sort.  At full size, where the
oracle's listing is too large to sort on the host, sampled sources are compared
row for row and every row's triangle and the uniqueness of rows are checked.
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


def _sorted_rows(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.int64).reshape(-1, 3)
    return a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))] if len(a) else a


def _gpu_listing(tc, n, s, d, *, order=0, offset_bytes=4, capacity=None, tune=None):
    p = tc.Pipeline(n, max(len(s), 1), offset_bytes=offset_bytes, order=order, tune=tune)
    p.build(_dev(s), _dev(d))
    p.orient()
    p.count()
    T = p.result().total
    p.list_triangles(T if capacity is None else capacity)
    return p, T


def _oracle_listing(n, s, d, order=0):
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    return oracle.list_triangles(dp, dc)


def _check_same(tc, n, s, d, order=0, offset_bytes=4, tune=None):
    p, T = _gpu_listing(tc, n, s, d, order=order, offset_bytes=offset_bytes, tune=tune)
    rows = p.listing().cpu().numpy()
    want = _oracle_listing(n, s, d, order)
    assert len(rows) == len(want) == T
    np.testing.assert_array_equal(_sorted_rows(rows), _sorted_rows(want))
    # sources come in increasing id order
    assert np.all(np.diff(rows[:, 0]) >= 0)


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_list_golden_fixtures(tc, fx):
    _say("list golden", fx.name)
    for order in (tc.TC_ORDER_DEGREE, tc.TC_ORDER_ID):
        for ob in (4, 8):
            p, _ = _gpu_listing(tc, fx.n, fx.src, fx.dst, order=order, offset_bytes=ob)
            rows = p.listing().cpu().numpy()
            assert sorted(tuple(sorted(r)) for r in rows.tolist()) == fx.triangle_sets
            _check_same(tc, fx.n, fx.src, fx.dst, order, ob)


def test_list_random_tiny(tc):
    for seed in range(40):
        rng = np.random.default_rng(500 + seed)
        n = int(rng.integers(1, 48))
        n, s, d = pins.random_simple(n, float(rng.choice([0.1, 0.3, 0.6, 1.0])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        _say("list tiny seed", seed, "n", n)
        for order in (0, 1):
            _check_same(tc, n, s, d, order, 4 + 4 * (seed % 2))


@pytest.mark.parametrize("scale,seed", [(10, 1), (14, 2), (16, 3)])
def test_list_rmat(tc, scale, seed):
    s, d, n = graphgen.rmat(scale, 16, seed)
    _say("list rmat", scale)
    for order in (0, 1):
        _check_same(tc, n, s.numpy(), d.numpy(), order)


def test_list_config1(tc):
    for seed in range(3):
        s, d, n = graphgen.erdos_renyi(1024, 8192, seed)
        _check_same(tc, n, s.numpy(), d.numpy())


def test_list_hub_beyond_one_slice_and_clique(tc):
    """Id order puts every vertex in N+(0) (several table slices, workgroup mode);
    K_120 under id order has sources of every out-degree."""
    rng = np.random.default_rng(11)
    n = 4001
    s = np.concatenate([np.zeros(4000, dtype=np.int64), rng.integers(1, n, 30000)])
    d = np.concatenate([np.arange(1, n), rng.integers(1, n, 30000)])
    for order in (0, 1):
        _check_same(tc, n, s, d, order)
    n, s, d = pins.complete(120)
    _check_same(tc, n, s, d, 1)


def test_list_with_split_sources(tc):
    """Equal-work quanta (tc_tune.split_log2) split the heavy sources of the counting pass;
    the rows of the writing pass (never split) must land in the same per-source ranges."""
    tune = {"split_log2": 3, "small_max": 16}
    s, d, n = graphgen.rmat(12, 16, 8)
    for order in (0, 1):
        _check_same(tc, n, s.numpy(), d.numpy(), order, tune=tune)
    n, s, d = pins.complete(60)
    _check_same(tc, n, s, d, 1, tune=tune)


@pytest.mark.parametrize("kicks", [-1, 1])
def test_list_probe_fallback_modes(tc, kicks):
    """Stash and sorted probe modes (tc_tune.max_kicks) write the same rows."""
    tune = {"max_kicks": kicks}
    s, d, n = graphgen.rmat(12, 16, 8)
    for order in (0, 1):
        _check_same(tc, n, s.numpy(), d.numpy(), order, tune=tune)
    n, s, d = pins.complete(60)
    _check_same(tc, n, s, d, 0, tune=tune)


def test_list_capacity_and_degenerate(tc):
    n, s, d = pins.complete(9)  # 84 triangles
    p, T = _gpu_listing(tc, n, s, d, capacity=100)
    assert T == 84 and len(p.listing()) == 84
    # too small: the count reports the error and no row is written
    p.triples.fill_(-7)
    p.list_triangles(83)
    torch.cuda.synchronize()
    assert int(p.list_count.item()) == -3
    assert int((p.triples != -7).sum().item()) == 0
    with pytest.raises(tc.TcError):
        p.listing()
    # exactly enough
    p.list_triangles(84)
    assert len(p.listing()) == 84
    # no triangles, no vertices, capacity 0
    for n, s, d in [(0, [], []), (1, [], []), (6, [0, 1, 2], [1, 2, 3]), (5, [2, 2], [2, 2])]:
        p, T = _gpu_listing(tc, n, s, d, capacity=0)
        assert T == 0 and len(p.listing()) == 0


def test_list_rmat_scale20_sampled(tc):
    """The benchmark graph: count, row uniqueness and every row's triangle on the GPU side,
    and the rows of sampled sources against the oracle's DAG row by row."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    p = tc.Pipeline(n, s.numel(), offset_bytes=4)
    p.enqueue(s, d)
    T = p.result().total
    p.list_triangles(T)
    rows = p.listing()
    _say("scale 20 listing", T)
    hs, hd = s.cpu().numpy(), d.cpu().numpy()
    rp, col = oracle.clean(n, hs, hd)
    dp, dc = oracle.orient(rp, col)
    assert oracle.count(dp, dc) == T == rows.shape[0]
    r = rows.to(torch.int64)
    assert bool((r[1:, 0] >= r[:-1, 0]).all())
    key = (r[:, 0] << 42) | (r[:, 1] << 21) | r[:, 2]
    assert torch.unique(key).numel() == T
    del key
    # every row is a closed wedge of the oracle's DAG: check membership by binary search
    dpt = torch.as_tensor(dp).cuda()
    dct = torch.as_tensor(dc.astype(np.int64)).cuda()
    rng = np.random.default_rng(7)
    pick = torch.as_tensor(rng.choice(T, size=min(T, 4_000_000), replace=False)).cuda()
    sr = r[pick]
    edge_key = torch.repeat_interleave(torch.arange(n, device="cuda"), dpt[1:] - dpt[:-1]) * n + dct
    for a, b in ((0, 1), (1, 2), (0, 2)):
        q = sr[:, a] * n + sr[:, b]
        at = torch.searchsorted(edge_key, q).clamp(max=edge_key.numel() - 1)
        assert bool((edge_key[at] == q).all()), (a, b)
    # sampled sources row for row
    src_hits = torch.bincount(r[:, 0], minlength=n).cpu().numpy()
    firsts = np.concatenate([[0], np.cumsum(src_hits)])
    cand = np.flatnonzero((dp[1:] - dp[:-1]) >= 2)
    for u in rng.choice(cand, size=300, replace=False).tolist():
        nu = dc[dp[u]:dp[u + 1]]
        want = []
        for v in nu.tolist():
            for w in np.intersect1d(nu, dc[dp[v]:dp[v + 1]], assume_unique=True).tolist():
                want.append((u, v, w))
        got = rows[firsts[u]:firsts[u + 1]].cpu().numpy()
        np.testing.assert_array_equal(_sorted_rows(got), _sorted_rows(np.array(want).reshape(-1, 3)))
