"""GPU parity of the labelled triangle query (tc_count_labelled: the triangles whose vertex
labels, as a multiset, equal the query's three labels) against the oracle.

Counts are integers, so the bar is equality: the count of every query, and the number of
DAG edges the label filter keeps (written out here from its definition: an edge is kept
when its two labels are a sub-multiset of the query's).
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


def _kept(dp, dc, lab, q):
    """DAG edges whose label pair is a sub-multiset of the query."""
    if dc.size == 0:
        return 0
    src = np.repeat(np.arange(dp.size - 1), np.diff(dp))
    lo = np.minimum(lab[src], lab[dc])
    hi = np.maximum(lab[src], lab[dc])
    a, b, c = sorted(q)
    fits = ((lo == a) & ((hi == b) | (hi == c))) | ((lo == b) & (hi == c))
    return int(fits.sum())


def _queries(k, extra=()):
    return list(itertools.combinations_with_replacement(range(k), 3)) + list(extra)


def _check(tc, n, s, d, lab, queries, *, order=0, offset_bytes=4):
    p = _pipe(tc, n, s, d, order=order, offset_bytes=offset_bytes)
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    lab = np.asarray(lab, dtype=np.int32)
    lab_d = _dev(lab) if n > 0 else torch.zeros(1, dtype=torch.int32, device="cuda")
    for q in queries:
        p.labelled(lab_d, q)
        got = p.labelled_count()
        assert got == oracle.count_labelled(dp, dc, lab, q), (q, order, offset_bytes)
        assert int(p.labelled_kept.item()) == _kept(dp, dc, lab, q), q
    return p


def test_labelled_golden_fixtures(tc):
    for fx in goldens.all_fixtures():
        _say("labelled golden", fx.name)
        lab = graphgen.vertex_labels(fx.n, 3, 7).numpy()
        for order in (0, 1):
            _check(tc, fx.n, fx.src, fx.dst, lab, _queries(3), order=order,
                   offset_bytes=4 + 4 * order)


def test_labelled_closed_forms(tc):
    # K_n with label classes of sizes a, b, c (labels shuffled over the ids)
    a, b, c = 5, 4, 3
    n, s, d = pins.complete(a + b + c)
    lab = np.array([0] * a + [1] * b + [2] * c, dtype=np.int32)
    lab = lab[np.random.default_rng(3).permutation(n)]
    p = _pipe(tc, n, s, d)
    lab_d = _dev(lab)
    for q, want in [((0, 0, 0), comb(a, 3)), ((0, 1, 0), comb(a, 2) * b),
                    ((1, 2, 2), b * comb(c, 2)), ((2, 1, 0), a * b * c), ((3, 0, 0), 0),
                    ((2, 2, 2), comb(c, 3))]:
        p.labelled(lab_d, q)
        assert p.labelled_count() == want, q
    # one label everywhere: every triangle
    p.labelled(_dev(np.full(n, -9, np.int32)), (-9, -9, -9))
    assert p.labelled_count() == comb(n, 3)
    # a wheel whose hub has its own label: every triangle is the hub and two rim vertices
    k = 9
    s = [0] * k + list(range(1, k + 1))
    d = list(range(1, k + 1)) + [i % k + 1 for i in range(1, k + 1)]
    lab = np.array([5] + [7] * k, dtype=np.int32)
    p = _pipe(tc, k + 1, s, d)
    for q, want in [((5, 7, 7), k), ((7, 7, 7), 0), ((5, 5, 7), 0)]:
        p.labelled(_dev(lab), q)
        assert p.labelled_count() == want, q


def test_labelled_random_tiny(tc):
    for seed in range(30):
        rng = np.random.default_rng(1700 + seed)
        n = int(rng.integers(1, 40))
        n, s, d = pins.random_simple(n, float(rng.choice([0.2, 0.5, 0.9])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        k = int(rng.integers(1, 4))
        lab = graphgen.vertex_labels(n, k, seed).numpy() - 1  # labels may be negative
        _say("labelled tiny seed", seed, "n", n, "k", k)
        qs = [tuple(x - 1 for x in q) for q in _queries(k, [(k, 0, 0), (0, k, k)])]
        for order in (0, 1):
            _check(tc, n, s, d, lab, qs, order=order, offset_bytes=4 + 4 * (seed % 2))


@pytest.mark.parametrize("scale,k,seed", [(10, 2, 1), (14, 3, 2), (16, 4, 3)])
def test_labelled_rmat(tc, scale, k, seed):
    s, d, n = graphgen.rmat(scale, 16, seed)
    lab = graphgen.vertex_labels(n, k, seed).numpy()
    _say("labelled rmat", scale, "k", k)
    for order in (0, 1):
        _check(tc, n, s.numpy(), d.numpy(), lab, _queries(k), order=order)


def test_labelled_capacity_and_degenerate(tc):
    from paper_1909_02127_amd import _lib
    n, s, d = pins.complete(8)  # 28 edges
    p = _pipe(tc, n, s, d)
    lab = _dev(np.zeros(n, np.int32))
    # a column capacity below m is reported on the device, and nothing is counted
    ws = torch.empty(_lib.tc_count_labelled_workspace(n, 27), dtype=torch.uint8, device="cuda")
    total = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    kept = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.tc_count_labelled(n, p.dag_ptr, p.dag_col[:27], lab, (0, 0, 0), total, ws,
                           kept_out=kept)
    torch.cuda.synchronize()
    assert int(kept.item()) == -_lib.TC_ERR_CAPACITY
    assert int(total.item()) == 0
    # the same buffers at the full capacity, without kept_out
    ws = torch.empty(_lib.tc_count_labelled_workspace(n, 28), dtype=torch.uint8, device="cuda")
    _lib.tc_count_labelled(n, p.dag_ptr, p.dag_col, lab, (0, 0, 0), total, ws)
    torch.cuda.synchronize()
    assert int(total.item()) == comb(8, 3)
    # a workspace below the query's size is refused on the host
    with pytest.raises(_lib.TcError):
        _lib.tc_count_labelled(n, p.dag_ptr, p.dag_col, lab, (0, 0, 0), total, ws[:100])
    for n, s, d in [(0, [], []), (1, [], []), (6, [0, 1, 2], [1, 2, 3]), (5, [2, 2], [2, 2]),
                    (3, [0, 1, 0], [1, 2, 2])]:
        lab = np.arange(n, dtype=np.int32) % 2
        _check(tc, n, s, d, lab, _queries(2))


def test_labelled_rmat_scale20_full(tc):
    """R-MAT scale 20, edge factor 16, four labels: a query of each shape against the
    oracle, and the counts of all 20 label multisets summing to the unlabelled total."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    lab = graphgen.vertex_labels(n, 4, 20, device="cuda")
    p = tc.Pipeline(n, s.numel(), offset_bytes=4)
    p.build(s, d)
    p.orient()
    p.count()
    T = p.result().total
    got = {}
    for q in _queries(4):
        p.labelled(lab, q)
        got[q] = p.labelled_count()
    assert sum(got.values()) == T
    _say("scale 20 labelled: oracle")
    hs, hd, hl = s.cpu().numpy(), d.cpu().numpy(), lab.cpu().numpy()
    rp, col = oracle.clean(n, hs, hd)
    dp, dc = oracle.orient(rp, col, 0)
    for q in [(0, 0, 0), (1, 1, 2), (0, 2, 2), (0, 1, 3)]:
        assert got[q] == oracle.count_labelled(dp, dc, hl, q), q
