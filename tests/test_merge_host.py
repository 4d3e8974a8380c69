"""Host emulation of the segmented merge-path intersection (the segmented-intersection
operator): the index arithmetic the merge kernel runs, checked on the CPU.

Every DAG edge e = (u, v) with d+(u) >= 2 and d+(v) >= 1 owns a stretch of the merge
space of length d+(u) + d+(v): the merge of A = N+(u) and B = N+(v).  An exclusive scan P
of those lengths lays the stretches end to end.  A wave takes 64 consecutive chunks of C
steps; lane l starts at base + l*C, finds its edge by a binary search of P inside the
wave's edge range, finds its place in that edge's merge by the merge-path diagonal search
(ties: A first), and merges sequentially, moving to the next edge with a non-empty stretch
at its end.  A match is counted when A[i] is taken while B's head equals it, so each
common out-neighbour w is found exactly once, in the chunk that takes A[i].  Support adds
one to (u, v), to (u, w) at A's position and to (v, w) at B's position.

The checks: every position is merged exactly once, no list is read out of its bounds, and
the count and the support equal the oracle's, for chunk sizes that do and do not divide
the stretches, on random, dense and degenerate graphs."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import pins

WAVE = 64
BIG = 2**31 - 1


def upper_bound(P, lo, hi, x):
    """First index in [lo, hi) with P[idx] > x (hi if none)."""
    while lo < hi:
        mid = (lo + hi) // 2
        if P[mid] <= x:
            lo = mid + 1
        else:
            hi = mid
    return lo


def merge_emulate(rp, col, C, R=None):
    """Chunks of C steps per lane; with R, an edge's steps inside a chunk go in rounds of R
    that restage both lists from the heads the previous round left (the kernel's LDS
    rounds), reading the R + 1 elements from each head clamped to its list."""
    rp = [int(x) for x in rp]
    col = [int(x) for x in col]
    n = len(rp) - 1
    m = rp[-1]
    d = [rp[u + 1] - rp[u] for u in range(n)]
    src_of = [u for u in range(n) for _ in range(d[u])]
    work = [(d[src_of[e]] + d[col[e]]) if d[src_of[e]] >= 2 and d[col[e]] >= 1 else 0
            for e in range(m)]
    P = [0]
    for w in work:
        P.append(P[-1] + w)
    S = P[-1]
    span = WAVE * C
    hits = 0
    sup = [0] * m
    merged = [0] * m

    def rd(lst_beg, idx, length):
        assert 0 <= idx < length  # the kernel guards every load the same way
        return col[lst_beg + idx]

    for base in range(0, S, span):
        e_lo = upper_bound(P, 0, m + 1, base) - 1
        e_hi = upper_bound(P, 0, m + 1, min(base + span, S) - 1) - 1
        assert 0 <= e_lo <= e_hi < m
        for lane in range(WAVE):
            p = base + lane * C
            if p >= S:
                continue
            pend = min(p + C, S)
            e = upper_bound(P, e_lo, e_hi + 2, p) - 1
            while True:
                assert e_lo <= e <= e_hi and P[e] <= p < P[e + 1]
                u, v = src_of[e], col[e]
                ab, a, bb, b = rp[u], d[u], rp[v], d[v]
                k = p - P[e]
                lo, hi = max(0, k - b), min(k, a)
                while lo < hi:
                    mid = (lo + hi) // 2
                    if rd(ab, mid, a) <= rd(bb, k - mid - 1, b):
                        lo = mid + 1
                    else:
                        hi = mid
                i, j = lo, k - lo
                av = rd(ab, i, a) if i < a else BIG
                bv = rd(bb, j, b) if j < b else BIG
                steps = min(pend, P[e + 1]) - p
                cuv = 0
                for t in range(steps):
                    if R and t % R == 0:
                        # a new round: stage A[i, i + R] and B[j, j + R] from the heads
                        for x in range(R + 1):
                            if a:
                                rd(ab, min(i + x, a - 1), a)
                            if b:
                                rd(bb, min(j + x, b - 1), b)
                        av = rd(ab, i, a) if i < a else BIG
                        bv = rd(bb, j, b) if j < b else BIG
                    if av <= bv:
                        if av == bv:
                            hits += 1
                            cuv += 1
                            sup[ab + i] += 1
                            sup[bb + j] += 1
                        i += 1
                        av = rd(ab, i, a) if i < a else BIG
                    else:
                        j += 1
                        bv = rd(bb, j, b) if j < b else BIG
                sup[e] += cuv
                merged[e] += steps
                p += steps
                if p >= pend:
                    break
                e = upper_bound(P, e + 1, e_hi + 2, p) - 1
    assert merged == work
    return hits, np.array(sup, dtype=np.uint64)


def _dag(n, s, d):
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    return oracle.orient(rp, col, oracle.ORDER_DEGREE)


def _check(n, s, d, chunks=(1, 3, 8, 64)):
    dp, dc = _dag(n, s, d)
    T, sup = oracle.edge_support(dp, dc)
    for C in chunks:
        h, s_ = merge_emulate(dp, dc, C)
        assert h == T, C
        np.testing.assert_array_equal(s_, sup)
    # the kernel's layout: 64-step chunks merged in rounds of 8
    h, s_ = merge_emulate(dp, dc, 64, R=8)
    assert h == T
    np.testing.assert_array_equal(s_, sup)


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 120))
    n, s, d = pins.random_simple(n, float(rng.choice([0.05, 0.2, 0.5])), seed)
    _check(n, s, d)


def test_dense_clique_and_id_order():
    n = 24
    s, d = zip(*[(i, j) for i in range(n) for j in range(i + 1, n)])
    _check(n, s, d, chunks=(1, 5, 64))
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, oracle.ORDER_ID)
    T, sup = oracle.edge_support(dp, dc)
    h, s_ = merge_emulate(dp, dc, 7)
    assert h == T == 24 * 23 * 22 // 6
    np.testing.assert_array_equal(s_, sup)


def test_rmat_small():
    s, d, n = graphgen.rmat(9, 8, 3)
    _check(n, s.numpy(), d.numpy(), chunks=(4, 64))


def test_degenerate():
    _check(1, [0], [0])            # no edges
    _check(3, [0, 1], [1, 2])      # a path: no stretch has work
    _check(3, [0, 1, 0], [1, 2, 2])  # one triangle
