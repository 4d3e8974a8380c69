"""GPU parity of the triangle query with edge labels (tc_edge_labels records each DAG edge's
label from the labelled input pairs; tc_count_edge_labelled keeps the edges whose label is in
the query and counts the triangles whose edge labels match the query's, in the count kernel
with the labels as per-edge codes) against the oracle.

Counts are integers, so the bar is equality.  The per-edge labels are compared with their
definition (the largest label of an edge's pairs), written out here from the pairs.  At scale
20 the oracle takes minutes per query, so the full-size test checks what holds at any size:
the counts of all 20 label multisets sum to the unlabelled total, and with one label
everywhere only that label's query counts, every triangle.
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


def _dev(x, dt=np.int32):
    return torch.as_tensor(np.asarray(x, dtype=dt)).cuda()


def _pipe(tc, n, s, d, lab, *, order=0, offset_bytes=4):
    p = tc.Pipeline(n, max(len(s), 1), offset_bytes=offset_bytes, order=order)
    sd, dd = _dev(s), _dev(d)
    p.build(sd, dd)
    p.orient()
    p.edge_labels(sd, dd, _dev(lab, np.uint8))
    return p


def _want_labels(dp, dc, s, d, lab):
    L = {}
    for a, b, x in zip(s, d, lab):
        a, b, x = int(a), int(b), int(x)
        if a != b:
            k = (min(a, b), max(a, b))
            L[k] = max(L.get(k, x), x)
    out = np.zeros(dc.size, dtype=np.uint8)
    for u in range(dp.size - 1):
        for e in range(dp[u], dp[u + 1]):
            v = int(dc[e])
            out[e] = L[(min(u, v), max(u, v))]
    return out


def _check(tc, n, s, d, lab, queries, *, order=0, offset_bytes=4, labels=True, tune=None):
    p = _pipe(tc, n, s, d, lab, order=order, offset_bytes=offset_bytes)
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    want_lab = _want_labels(dp, dc, s, d, lab)
    if labels:
        torch.cuda.synchronize()
        assert int(p.edge_label_m.item()) == dc.size
        np.testing.assert_array_equal(p.edge_label[: dc.size].cpu().numpy(), want_lab)
    for q in queries:
        p.edge_labelled(q, tune=tune)
        assert p.edge_labelled_count() == oracle.count_edge_labelled(dp, dc, s, d, lab, q), \
            (q, order, offset_bytes)
        # the filter keeps the edges whose label is one of the query's
        assert int(p.edge_labelled_kept.item()) == int(np.isin(want_lab, q).sum()), q
    return p


def test_edge_labelled_random_tiny(tc):
    for seed in range(12):
        rng = np.random.default_rng(3100 + seed)
        n = int(rng.integers(3, 30))
        n, s, d = pins.random_simple(n, float(rng.choice([0.2, 0.5, 0.9])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        lab = rng.integers(0, 4, size=len(s))
        _say("edge-labelled tiny seed", seed, "n", n)
        queries = list(itertools.product(range(4), repeat=3))
        _check(tc, n, s, d, lab, queries, order=seed % 2, offset_bytes=4 + 4 * (seed // 6))


def test_edge_labelled_golden_and_closed_forms(tc):
    for fx in goldens.all_fixtures():
        lab = np.arange(len(fx.src)) % 3
        for order in (0, 1):
            _check(tc, fx.n, fx.src, fx.dst, lab, [(0, 0, 0), (0, 1, 2), (1, 1, 2)], order=order,
                   offset_bytes=4 + 4 * order)
    # K_n with edge {i, j} labelled (i + j) mod 2
    n = 13
    s = np.array([i for i in range(n) for j in range(i + 1, n)])
    d = np.array([j for i in range(n) for j in range(i + 1, n)])
    p = _pipe(tc, n, s, d, (s + d) % 2)
    e, o = (n + 1) // 2, n // 2
    for q, want in [((0, 0, 0), comb(e, 3) + comb(o, 3)),
                    ((1, 0, 1), comb(e, 2) * o + comb(o, 2) * e), ((1, 1, 1), 0), ((0, 0, 1), 0)]:
        p.edge_labelled(q)
        assert p.edge_labelled_count() == want, q


def test_edge_labelled_rmat_and_probe_modes(tc):
    from paper_1909_02127_amd import _lib
    s, d, n = graphgen.rmat(11, 16, 8)
    s, d = s.numpy(), d.numpy()
    lab = np.random.default_rng(8).integers(0, 4, size=s.size)
    tunes = [None, _lib.make_tune(probe=_lib.TC_PROBE_SORTED), _lib.make_tune(max_kicks=1),
             _lib.make_tune(small_max=1), _lib.make_tune(split_log2=8)]
    for order in (0, 1):
        for i, tune in enumerate(tunes):
            _say("edge-labelled rmat 11 order", order, "tune", i)
            _check(tc, n, s, d, lab, [(0, 0, 0), (0, 1, 3), (2, 2, 1)], order=order,
                   labels=i == 0, tune=tune)


def test_edge_labelled_errors(tc):
    from paper_1909_02127_amd import _lib
    n, s, d = 5, [0, 1, 2], [1, 2, 0]
    p = _pipe(tc, n, s, d, [1, 1, 1])
    p.edge_labelled((1, 1, 1))
    assert p.edge_labelled_count() == 1
    p.edge_labels(_dev(s), _dev(d), _dev([1, 4, 1], np.uint8))  # a label above 3
    with pytest.raises(_lib.TcError):
        p.edge_labelled_count()
    p.edge_labels(_dev([0, 3]), _dev([1, 4]), _dev([0, 0], np.uint8))  # not a DAG edge
    with pytest.raises(_lib.TcError):
        p.edge_labelled_count()
    with pytest.raises(_lib.TcError):
        p.edge_labelled((0, 4, 0))  # a query label above 3, refused on the host


def test_edge_labelled_rmat_scale20_full(tc):
    """R-MAT scale 20 with four uniform edge labels: the counts of all 20 label multisets
    sum to the triangle count; one label everywhere gives every triangle."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    lab = torch.as_tensor(np.random.default_rng(20).integers(0, 4, size=s.numel()),
                          dtype=torch.uint8).cuda()
    p = tc.Pipeline(n, s.numel(), offset_bytes=4)
    p.build(s, d)
    p.orient()
    p.count()
    T = p.result().total
    p.edge_labels(s, d, lab)
    got = {}
    for q in itertools.combinations_with_replacement(range(4), 3):
        p.edge_labelled(q)
        got[q] = p.edge_labelled_count()
    assert sum(got.values()) == T
    # one label everywhere: every triangle, under that label only
    p.edge_labels(s, d, torch.full_like(lab, 2))
    p.edge_labelled((2, 2, 2))
    assert p.edge_labelled_count() == T
    p.edge_labelled((2, 2, 1))
    assert p.edge_labelled_count() == 0


def test_edge_labelled_degenerate(tc):
    from paper_1909_02127_amd import _lib
    for n, s, d in [(0, [], []), (1, [], []), (3, [0, 0], [0, 0]), (4, [0, 1], [1, 2]),
                    (3, [0, 1, 0], [1, 2, 2])]:
        lab = np.arange(len(s)) % 4
        _check(tc, n, np.array(s, np.int32), np.array(d, np.int32), lab,
               [(0, 0, 0), (0, 1, 2), (3, 3, 3)])
    # a column capacity below m is reported on the device, and nothing is counted
    n, s, d = pins.complete(6)  # 15 edges
    p = _pipe(tc, n, s, d, np.zeros(len(s), np.int64))
    ws = torch.empty(_lib.tc_count_edge_labelled_workspace(n, 14), dtype=torch.uint8,
                     device="cuda")
    total = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    kept = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.tc_count_edge_labelled(n, p.dag_ptr, p.dag_col[:14], p.edge_label, (0, 0, 0), total, ws,
                                kept_out=kept)
    torch.cuda.synchronize()
    assert int(kept.item()) == -_lib.TC_ERR_CAPACITY and int(total.item()) == 0
    p.edge_labelled((0, 0, 0))
    assert p.edge_labelled_count() == comb(6, 3)
