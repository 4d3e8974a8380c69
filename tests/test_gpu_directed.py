"""GPU parity of the directed triangle query (tc_edge_directions records each DAG edge's
arcs; tc_count_directed counts the matches of a three-node digraph with every pair joined,
induced or not) against the oracle.

Counts are integers, so the bar is equality.  The direction bytes are compared with their
definition (bit 0: the arc from the row's vertex to the column, bit 1: the reverse), written
out here from the arc set.  At scale 20 the oracle is too slow for every query, so the full-
size test checks what holds at any size: the seven induced classes partition the triangles,
reversing every arc and the query changes nothing, and with every arc reciprocal the
all-arcs query counts the undirected triangles.
"""
from __future__ import annotations

import itertools
import sys
from math import comb

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests import goldens

pytestmark = pytest.mark.gpu

CYCLE = (1, 2, 1)   # 0 -> 1 -> 2 -> 0
FFL = (1, 1, 1)     # 0 -> 1, 0 -> 2, 1 -> 2
ALL = (3, 3, 3)
SWAP = {1: 2, 2: 1, 3: 3}


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


def _classes():
    """One query of each of the 7 isomorphism classes."""
    out = {}
    for codes in itertools.product((1, 2, 3), repeat=3):
        arcs = set()
        for (i, j), c in zip(((0, 1), (0, 2), (1, 2)), codes):
            if c & 1:
                arcs.add((i, j))
            if c & 2:
                arcs.add((j, i))
        key = min(tuple(sorted((p[i], p[j]) for i, j in arcs))
                  for p in itertools.permutations(range(3)))
        out.setdefault(key, codes)
    assert len(out) == 7
    return list(out.values())


def _pipe(tc, n, s, d, *, order=0, offset_bytes=4):
    p = tc.Pipeline(n, max(len(s), 1), offset_bytes=offset_bytes, order=order)
    sd, dd = _dev(s), _dev(d)
    p.build(sd, dd)
    p.orient()
    p.edge_directions(sd, dd)
    return p


def _want_dir(dp, dc, s, d):
    A = {(int(a), int(b)) for a, b in zip(s, d) if a != b}
    out = np.zeros(dc.size, dtype=np.uint8)
    for u in range(dp.size - 1):
        for e in range(dp[u], dp[u + 1]):
            v = int(dc[e])
            out[e] = int((u, v) in A) | 2 * int((v, u) in A)
    return out


def _check(tc, n, s, d, queries, *, order=0, offset_bytes=4, dirs=True):
    p = _pipe(tc, n, s, d, order=order, offset_bytes=offset_bytes)
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    if dirs:
        torch.cuda.synchronize()
        assert int(p.direction_m.item()) == dc.size
        np.testing.assert_array_equal(p.direction[: dc.size].cpu().numpy(),
                                      _want_dir(dp, dc, s, d))
    for q in queries:
        for induced in (False, True):
            p.directed(q, induced=induced)
            got = p.directed_count()
            want = oracle.count_directed(dp, dc, s, d, q, induced=induced)
            assert got == want, (q, induced, order, offset_bytes)
    return p


def _random_digraph(n, prob, seed):
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < prob
    np.fill_diagonal(a, False)
    s, d = np.nonzero(a)
    extra = rng.integers(0, max(n, 1), size=(2, 3))
    s = np.concatenate([s, s[:2], extra[0], extra[0]])
    d = np.concatenate([d, d[:2], extra[0], extra[1]])
    return s.astype(np.int32), d.astype(np.int32)


def test_directed_all_queries_random_tiny(tc):
    for seed in range(12):
        rng = np.random.default_rng(2100 + seed)
        n = int(rng.integers(3, 24))
        s, d = _random_digraph(n, float(rng.choice([0.2, 0.5, 0.8])), seed)
        _say("directed tiny seed", seed, "n", n)
        queries = list(itertools.product((1, 2, 3), repeat=3))
        _check(tc, n, s, d, queries, order=seed % 2, offset_bytes=4 + 4 * (seed // 6))


def test_directed_golden_fixtures(tc):
    # the fixtures' pairs read as arcs, as listed
    for fx in goldens.all_fixtures():
        _say("directed golden", fx.name)
        for order in (0, 1):
            _check(tc, fx.n, fx.src, fx.dst, [CYCLE, FFL, ALL, (3, 1, 1)], order=order,
                   offset_bytes=4 + 4 * order)


def test_directed_closed_forms(tc):
    for seed, n in ((1, 6), (2, 17), (3, 40)):
        rng = np.random.default_rng(seed)
        iu, ju = np.triu_indices(n, 1)
        flip = rng.random(iu.size) < 0.5
        s, d = np.where(flip, ju, iu), np.where(flip, iu, ju)
        perm = rng.permutation(n)
        s, d = perm[s].astype(np.int32), perm[d].astype(np.int32)
        trans = sum(comb(int(o), 2) for o in np.bincount(s, minlength=n))
        p = _pipe(tc, n, s, d)
        for induced in (False, True):
            p.directed(FFL, induced=induced)
            assert p.directed_count() == trans
            p.directed(CYCLE, induced=induced)
            assert p.directed_count() == comb(n, 3) - trans
            p.directed(ALL, induced=induced)
            assert p.directed_count() == 0
    n = 9
    s = np.array([i for i in range(n) for j in range(n) if i != j], dtype=np.int32)
    d = np.array([j for i in range(n) for j in range(n) if i != j], dtype=np.int32)
    p = _pipe(tc, n, s, d)
    for q, induced, want in [(CYCLE, False, 2 * comb(n, 3)), (FFL, False, 6 * comb(n, 3)),
                             (ALL, False, comb(n, 3)), (CYCLE, True, 0), (ALL, True, comb(n, 3))]:
        p.directed(q, induced=induced)
        assert p.directed_count() == want, (q, induced)


@pytest.mark.parametrize("scale,seed", [(10, 1), (12, 2)])
def test_directed_rmat(tc, scale, seed):
    s, d, n = graphgen.rmat(scale, 16, seed)
    s, d = s.numpy(), d.numpy()
    _say("directed rmat", scale)
    for order in (0, 1):
        _check(tc, n, s, d, [CYCLE, FFL, (3, 1, 2), ALL] if scale <= 10 else [CYCLE, FFL],
               order=order, dirs=scale <= 10)


def test_directed_errors_and_degenerate(tc):
    from paper_1909_02127_amd import _lib
    n = 6
    s, d = np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32)
    p = _pipe(tc, n, s, d)
    # an arc whose pair is not an edge of this DAG
    p.edge_directions(_dev([0, 3]), _dev([1, 4]))
    with pytest.raises(_lib.TcError):
        p.directed_count()
    # an id out of range
    p.edge_directions(_dev([0, 9]), _dev([1, 2]))
    with pytest.raises(_lib.TcError):
        p.directed_count()
    p.edge_directions(_dev(s), _dev(d))
    p.directed(CYCLE)
    assert p.directed_count() == 1
    # codes outside 1..3 are refused on the host
    with pytest.raises(_lib.TcError):
        p.directed((0, 1, 1))
    # a workspace below the query's size is refused on the host
    ws = torch.empty(_lib.tc_count_directed_workspace(n), dtype=torch.uint8, device="cuda")
    total = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    with pytest.raises(_lib.TcError):
        _lib.tc_count_directed(n, p.dag_ptr, p.dag_col, p.direction, CYCLE, total, ws[:64])
    _lib.tc_count_directed(n, p.dag_ptr, p.dag_col, p.direction, CYCLE, total, ws)
    torch.cuda.synchronize()
    assert int(total.item()) == 1
    # a column capacity below m when recording the directions
    m_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.tc_edge_directions(n, p.dag_ptr, p.dag_col[:2], _dev(s), _dev(d), p.direction, m_out)
    torch.cuda.synchronize()
    assert int(m_out.item()) == -_lib.TC_ERR_CAPACITY
    for n, s, d in [(1, [], []), (3, [0, 0], [0, 0]), (4, [0, 1], [1, 2]), (3, [0, 1, 0], [1, 2, 2])]:
        _check(tc, n, np.array(s, np.int32), np.array(d, np.int32), [CYCLE, FFL, ALL])


def test_directed_rmat_scale20_full(tc):
    """R-MAT scale 20 (edge factor 16) read as arcs: the seven induced classes sum to the
    triangle count, reversal symmetry, and the all-reciprocal graph's all-arcs count."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    p = tc.Pipeline(n, 2 * s.numel(), offset_bytes=4)
    p.build(s, d)
    p.orient()
    p.count()
    T = p.result().total
    p.edge_directions(s, d)
    got = {}
    for q in _classes():
        p.directed(q, induced=True)
        got[q] = p.directed_count()
    _say("scale 20 directed classes", got)
    assert sum(got.values()) == T
    nonind = {}
    for q in (CYCLE, FFL, (3, 1, 1)):
        p.directed(q)
        nonind[q] = p.directed_count()
    # the reversed arcs
    p.edge_directions(d, s)
    for q in list(got)[:4]:
        p.directed(tuple(SWAP[x] for x in q), induced=True)
        assert p.directed_count() == got[q], q
    for q in nonind:
        p.directed(tuple(SWAP[x] for x in q))
        assert p.directed_count() == nonind[q], q
    # every arc reciprocal
    s2, d2 = torch.cat([s, d]), torch.cat([d, s])
    p.build(s2, d2)
    p.orient()
    p.edge_directions(s2, d2)
    p.directed(ALL)
    assert p.directed_count() == T
    p.directed(CYCLE, induced=True)
    assert p.directed_count() == 0


def test_directed_probe_modes_and_splits(tc):
    """Every probe structure of the count kernel (cuckoo, stash, sorted, the in-memory
    search of very long rows), both source paths and split sources give the oracle's
    counts: the direction code of (u, w) follows its key wherever the key sits."""
    from paper_1909_02127_amd import _lib
    s, d, n = graphgen.rmat(11, 16, 5)
    s, d = s.numpy(), d.numpy()
    # a hub adjacent to everything: in id order its out-list is searched in memory
    rng = np.random.default_rng(8)
    hn = 4001
    hs = np.concatenate([np.zeros(4000, np.int64), rng.integers(1, hn, 30000)])
    hd = np.concatenate([np.arange(1, hn), rng.integers(1, hn, 30000)])
    flip = rng.random(hs.size) < 0.5
    hs, hd = np.where(flip, hd, hs).astype(np.int32), np.where(flip, hs, hd).astype(np.int32)
    tunes = [_lib.make_tune(probe=_lib.TC_PROBE_SORTED), _lib.make_tune(max_kicks=1),
             _lib.make_tune(small_max=1), _lib.make_tune(split_log2=8),
             _lib.make_tune(small_max=96, split_log2=-1)]
    for n_, s_, d_ in ((n, s, d), (hn, hs, hd)):
        for order in (0, 1):
            p = _pipe(tc, n_, s_, d_, order=order)
            rp, col = oracle.clean(n_, s_, d_)
            dp, dc = oracle.orient(rp, col, order)
            want = {q: oracle.count_directed(dp, dc, s_, d_, q) for q in (CYCLE, FFL)}
            for i, tune in enumerate(tunes):
                for q in (CYCLE, FFL):
                    p.directed(q, tune=tune)
                    assert p.directed_count() == want[q], (n_, order, i, q)
