"""GPU parity of the paper's own pipeline: the NE filter (tc_ne_filter) against the
oracle's k-core, and the materialised two-iteration advance (tc_count_bfs) against
the oracle's count and listing, with and without the filter, in both orders."""
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


def _pipeline(tc, n, s, d, order=0, offset_bytes=4):
    p = tc.Pipeline(n, max(len(s), 1), offset_bytes=offset_bytes, order=order)
    p.build(_dev(s), _dev(d))
    p.orient()
    torch.cuda.synchronize()
    return p


def _ne(tc, p, rounds=64, k=2):
    from paper_1909_02127_amd import _lib
    keep = torch.zeros(max(p.n, 1), dtype=torch.uint8, device="cuda")
    stats = torch.zeros(3, dtype=torch.int64, device="cuda")
    ws = torch.empty(_lib.tc_ne_filter_workspace(p.n, rounds), dtype=torch.uint8, device="cuda")
    _lib.tc_ne_filter(p.n, p.row_ptr, p.col, keep, stats, ws, min_degree=k, max_rounds=rounds)
    torch.cuda.synchronize()
    return keep[: p.n].cpu().numpy(), stats.cpu().numpy()


def _bfs(tc, p, keep=None, with_rows=True):
    from paper_1909_02127_amd import _lib
    cap = p.dag_col.numel()
    ws = torch.empty(_lib.tc_count_bfs_workspace(p.n, cap), dtype=torch.uint8, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    kp = None if keep is None else torch.as_tensor(keep, dtype=torch.uint8).cuda()
    rows = None
    if with_rows:
        p.count()
        T = p.result().total
        rows = torch.full((max(T, 1), 3), -1, dtype=torch.int32, device="cuda")
    _lib.tc_count_bfs(p.n, p.dag_ptr, p.dag_col, stats, ws, frontier_capacity=cap, keep=kp,
                      matches=rows, total=total)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    out = None
    if rows is not None:
        out = rows[: int(st[2])].cpu().numpy()
    return st, int(total.item()), out


def _sorted_rows(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 3)
    return a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))] if len(a) else a


def _frontier_by_definition(dp, dc, keep=None):
    """Partial matches after iteration 1 and the candidate wedges of iteration 2."""
    n = dp.size - 1
    dplus = np.diff(dp)
    ok_v = np.ones(n, dtype=bool) if keep is None else keep.astype(bool)
    F = 0
    W = 0
    for u in range(n):
        if dplus[u] < 2 or not ok_v[u]:
            continue
        for v in dc[dp[u]:dp[u + 1]]:
            if ok_v[v] and dplus[v] >= 1:
                F += 1
                W += int(dplus[v])
    return F, W


def _check(tc, n, s, d, order=0, offset_bytes=4, rounds=64):
    p = _pipeline(tc, n, s, d, order, offset_bytes)
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    T = oracle.count(dp, dc)
    want_rows = _sorted_rows(oracle.list_triangles(dp, dc))
    # the NE filter against the oracle's 2-core
    keep, nst = _ne(tc, p, rounds)
    core = oracle.kcore(rp, col, 2)
    if n > 0:
        assert nst[2] == 1  # converged
        np.testing.assert_array_equal(keep, core)
        assert nst[0] == int(core.sum())
    for kp in (None, keep if n > 0 else None):
        st, total, rows = _bfs(tc, p, kp)
        assert st[3] == 0 and st[2] == T == total
        if n <= 3000:
            F, W = _frontier_by_definition(dp, dc, kp)
            assert (st[0], st[1]) == (F, W)
        np.testing.assert_array_equal(_sorted_rows(rows), want_rows)


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_bfs_golden_fixtures(tc, fx):
    _say("bfs golden", fx.name)
    for order in (0, 1):
        _check(tc, fx.n, fx.src, fx.dst, order, 4 + 4 * order)


def test_bfs_random_tiny(tc):
    for seed in range(30):
        rng = np.random.default_rng(1300 + seed)
        n = int(rng.integers(1, 60))
        n, s, d = pins.random_simple(n, float(rng.choice([0.03, 0.08, 0.2, 0.5])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        _say("bfs tiny seed", seed, "n", n)
        for order in (0, 1):
            _check(tc, n, s, d, order, 4 + 4 * (seed % 2))


@pytest.mark.parametrize("scale,seed", [(10, 1), (14, 2)])
def test_bfs_rmat(tc, scale, seed):
    s, d, n = graphgen.rmat(scale, 16, seed)
    _say("bfs rmat", scale)
    for order in (0, 1):
        _check(tc, n, s.numpy(), d.numpy(), order)


def test_bfs_peel_chains_and_rounds(tc):
    """A triangle with a long pendant path peels one path vertex per round at worst: with
    few rounds the filter keeps a superset of the core and the count is unchanged."""
    n = 3 + 40
    s = [0, 1, 2] + list(range(2, 2 + 40))
    d = [1, 2, 0] + list(range(3, 3 + 40))
    p = _pipeline(tc, n, s, d)
    keep, st = _ne(tc, p, rounds=2)
    assert keep[:3].all() and st[0] == keep.sum() >= 3
    bst, total, _ = _bfs(tc, p, keep, with_rows=False)
    assert total == 1 and bst[3] == 0
    keep, st = _ne(tc, p, rounds=64)
    assert st[2] == 1 and keep.tolist() == [1, 1, 1] + [0] * 40


def test_bfs_capacity_and_empty(tc):
    from paper_1909_02127_amd import _lib
    n, s, d = pins.complete(7)
    p = _pipeline(tc, n, s, d)
    ws = torch.empty(_lib.tc_count_bfs_workspace(n, 5), dtype=torch.uint8, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    _lib.tc_count_bfs(n, p.dag_ptr, p.dag_col, stats, ws, frontier_capacity=5)
    torch.cuda.synchronize()
    assert int(stats[3].item()) == _lib.TC_ERR_CAPACITY
    rows = torch.zeros((10, 3), dtype=torch.int32, device="cuda")
    ws = torch.empty(_lib.tc_count_bfs_workspace(n, 21), dtype=torch.uint8, device="cuda")
    _lib.tc_count_bfs(n, p.dag_ptr, p.dag_col, stats, ws, frontier_capacity=21, matches=rows)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    assert st[2] == 35 and st[3] == _lib.TC_ERR_CAPACITY
    for n, s, d in [(0, [], []), (1, [], []), (6, [0, 1, 2], [1, 2, 3])]:
        _check(tc, n, s, d)


def test_bfs_rmat_scale20_count(tc):
    """The benchmark graph in id order (the paper's order): count and filter sizes."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    p = tc.Pipeline(n, s.numel(), offset_bytes=4, order=tc.TC_ORDER_ID)
    p.build(s, d)
    p.orient()
    p.count()
    T = p.result().total
    keep, nst = _ne(tc, p)
    st, total, _ = _bfs(tc, p, keep, with_rows=False)
    rp, col = oracle.clean(n, s.cpu().numpy(), d.cpu().numpy())
    np.testing.assert_array_equal(keep, oracle.kcore(rp, col, 2))
    dp, dc = oracle.orient(rp, col, oracle.ORDER_ID)
    assert total == T == oracle.count(dp, dc) and st[3] == 0
    _say("scale 20 id order: frontier", st[0], "candidate wedges", st[1], "matches", st[2])
