"""Pins for the CPU oracle (no GPU).

The oracle is checked against results that do not come from itself:
brute force over vertex triples, trace(A^3)/6 and diag(A^3)/2, closed forms of
graph families, invariants of the definition, and the golden fixtures.
"""
from __future__ import annotations

import numpy as np
import pytest

import graphgen
import oracle
from tests import goldens, pins


def _run(n, s, d, order=oracle.ORDER_DEGREE):
    return oracle.triangles(n, s, d, per_vertex=True, order=order)


@pytest.mark.parametrize("case", pins.closed_form_cases(), ids=lambda c: c[0])
def test_closed_forms(case):
    name, (n, s, d), T, t = case
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        total, per = _run(n, s, d, order)
        assert total == T, name
        assert int(per.sum()) == 3 * T
        if t is not None:
            np.testing.assert_array_equal(per, t)


@pytest.mark.parametrize("seed", range(120))
def test_brute_force_random_tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 33))
    p = float(rng.choice([0.05, 0.15, 0.3, 0.5, 0.8, 1.0]))
    n, s, d = pins.random_simple(n, p, seed)
    bt, bper = pins.brute_force(n, s, d)
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        total, per = _run(n, s, d, order)
        assert total == bt
        np.testing.assert_array_equal(per, bper)


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_noisy_input(seed):
    """Duplicates, reversed pairs and self-loops do not change the counts."""
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(2, 28))
    n, s, d = pins.random_simple(n, float(rng.uniform(0.1, 0.9)), seed)
    bt, bper = pins.brute_force(n, s, d)
    n, s2, d2 = pins.noisy(n, s, d, seed)
    total, per = _run(n, s2, d2)
    assert total == bt
    np.testing.assert_array_equal(per, bper)


@pytest.mark.parametrize("seed", range(10))
def test_trace_a3_config1(seed):
    """G(1024, 8192), the small configuration itself, against trace(A^3)/6."""
    s, d, n = graphgen.erdos_renyi(1024, 8192, seed)
    tt, tper = pins.trace_cube(n, s.numpy(), d.numpy())
    total, per = _run(n, s.numpy(), d.numpy())
    assert total == tt
    np.testing.assert_array_equal(per, tper)


@pytest.mark.parametrize("seed", range(6))
def test_trace_a3_small_rmat(seed):
    """Skewed R-MAT graphs (hubs, duplicates, self-loops in the raw pairs)."""
    s, d, n = graphgen.rmat(9, 8, 300 + seed)
    tt, tper = pins.trace_cube(n, s.numpy(), d.numpy())
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        total, per = _run(n, s.numpy(), d.numpy(), order)
        assert total == tt
        np.testing.assert_array_equal(per, tper)


def test_clean_matches_set_definition():
    for seed in range(30):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 40))
        p = int(rng.integers(0, 120))
        s = rng.integers(0, n, p)
        d = rng.integers(0, n, p)
        row_ptr, col = oracle.clean(n, s, d)
        E = pins.edge_set(s, d)
        want = [sorted({b for e in E if a in e for b in e if b != a}) for a in range(n)]
        assert row_ptr[0] == 0 and row_ptr[-1] == 2 * len(E)
        for a in range(n):
            assert list(col[row_ptr[a]:row_ptr[a + 1]]) == want[a]


def test_clean_rejects_out_of_range():
    with pytest.raises(oracle.OracleError):
        oracle.clean(4, [0, 1], [2, 4])
    with pytest.raises(oracle.OracleError):
        oracle.clean(4, [-1], [2])


def test_orient_matches_definition():
    for seed in range(20):
        rng = np.random.default_rng(50 + seed)
        n, s, d = pins.random_simple(int(rng.integers(2, 30)), 0.4, seed)
        row_ptr, col = oracle.clean(n, s, d)
        deg = np.diff(row_ptr)
        key = rng.integers(0, 5, n)
        for order, rank in [(oracle.ORDER_DEGREE, lambda v: (deg[v], v)),
                            (oracle.ORDER_ID, lambda v: v),
                            (oracle.ORDER_KEY, lambda v: (key[v], v))]:
            dp, dc = oracle.orient(row_ptr, col, order, key)
            assert dp[-1] == row_ptr[-1] // 2
            for u in range(n):
                nbrs = col[row_ptr[u]:row_ptr[u + 1]]
                want = [v for v in nbrs if rank(u) < rank(v)]
                assert list(dc[dp[u]:dp[u + 1]]) == want


def test_orientation_order_invariance():
    s, d, n = graphgen.rmat(11, 8, 5)
    row_ptr, col = oracle.clean(n, s.numpy(), d.numpy())
    results = []
    rng = np.random.default_rng(3)
    for order, key in [(oracle.ORDER_DEGREE, None), (oracle.ORDER_ID, None),
                       (oracle.ORDER_KEY, rng.integers(0, 1 << 40, n))]:
        dp, dc = oracle.orient(row_ptr, col, order, key)
        results.append(oracle.count(dp, dc, per_vertex=True))
    for total, per in results[1:]:
        assert total == results[0][0]
        np.testing.assert_array_equal(per, results[0][1])
    assert int(results[0][1].sum()) == 3 * results[0][0]


def test_relabel_invariance():
    s, d, n = graphgen.rmat(10, 8, 9)
    s, d = s.numpy(), d.numpy()
    total, per = _run(n, s, d)
    perm = np.random.default_rng(1).permutation(n)
    total2, per2 = _run(n, perm[s], perm[d])
    assert total2 == total
    np.testing.assert_array_equal(per2[perm], per)


def test_disjoint_union_additive():
    parts = [pins.complete(7), pins.wheel(6), pins.petersen(), pins.friendship(4)]
    s_all, d_all, off, T, pers = [], [], 0, 0, []
    for n, s, d in parts:
        s_all += [x + off for x in s]
        d_all += [x + off for x in d]
        off += n
        t, p = _run(n, s, d)
        T += t
        pers.append(p)
    total, per = _run(off, s_all, d_all)
    assert total == T
    np.testing.assert_array_equal(per, np.concatenate(pers))


def test_vertex_triangles_definition():
    for seed in range(15):
        rng = np.random.default_rng(900 + seed)
        n, s, d = pins.random_simple(int(rng.integers(3, 30)), 0.35, seed)
        n, s, d = pins.noisy(n, s, d, seed)
        _, bper = pins.brute_force(n, s, d)
        for v in range(n):
            assert oracle.vertex_triangles(n, s, d, v) == int(bper[v])


def test_threads_do_not_change_counts():
    s, d, n = graphgen.rmat(12, 16, 77)
    rp, c = oracle.clean(n, s.numpy(), d.numpy())
    dp, dc = oracle.orient(rp, c)
    a = oracle.count(dp, dc, per_vertex=True, threads=1)
    b = oracle.count(dp, dc, per_vertex=True, threads=4)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_golden_fixtures(fx):
    """Hand-checked graphs, each with the closed form or fact that fixes its counts."""
    assert int(fx.per_vertex.sum()) == 3 * fx.triangles  # the fixture itself is consistent
    bt, bper = pins.brute_force(fx.n, fx.src, fx.dst)
    assert bt == fx.triangles
    np.testing.assert_array_equal(bper, fx.per_vertex)
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        total, per = _run(fx.n, fx.src, fx.dst, order)
        assert total == fx.triangles
        np.testing.assert_array_equal(per, fx.per_vertex)


def test_golden_config1_counts_pinned_by_trace():
    """The stored G(1024, 8192) counts agree with trace(A^3)/6 recomputed here."""
    import json
    import os
    with open(os.path.join(goldens.GOLDEN_DIR, "er1024_8192.json")) as f:
        data = json.load(f)
    for seed, g in data["graphs"].items():
        s, d, n = graphgen.erdos_renyi(1024, 8192, int(seed))
        tt, tper = pins.trace_cube(n, s.numpy(), d.numpy())
        assert g["triangles"] == tt
        np.testing.assert_array_equal(np.array(g["per_vertex"], dtype=np.uint64), tper)


# -- the listing M (triangle triples) ------------------------------------------------------


def _listing(n, s, d, order=oracle.ORDER_DEGREE):
    rp, col = oracle.clean(n, s, d)
    dp, dc = oracle.orient(rp, col, order)
    return dp, dc, oracle.list_triangles(dp, dc)


def _dag_edges(dp, dc):
    return {(u, int(v)) for u in range(dp.size - 1) for v in dc[dp[u]:dp[u + 1]]}


def _check_listing_shape(dp, dc, lst):
    """Every row is a wedge u -> v -> w closed by u -> w; rows are strictly increasing."""
    edges = _dag_edges(dp, dc)
    for u, v, w in lst.tolist():
        assert (u, v) in edges and (v, w) in edges and (u, w) in edges
    if len(lst) > 1:
        keys = [tuple(r) for r in lst.tolist()]
        assert all(a < b for a, b in zip(keys, keys[1:]))


@pytest.mark.parametrize("seed", range(60))
def test_list_brute_force_random_tiny(seed):
    """The listed vertex sets are exactly the brute-force triangles, once each."""
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(1, 30))
    n, s, d = pins.random_simple(n, float(rng.choice([0.1, 0.3, 0.6, 1.0])), seed)
    want = pins.brute_force_sets(n, s, d)
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        dp, dc, lst = _listing(n, s, d, order)
        assert sorted(tuple(sorted(r)) for r in lst.tolist()) == want
        _check_listing_shape(dp, dc, lst)


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_list_golden_fixtures(fx):
    """Hand-derived triangle sets of the fixtures (each from the fact its header states)."""
    assert len(fx.triangle_sets) == fx.triangles
    assert pins.brute_force_sets(fx.n, fx.src, fx.dst) == fx.triangle_sets
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        dp, dc, lst = _listing(fx.n, fx.src, fx.dst, order)
        assert sorted(tuple(sorted(r)) for r in lst.tolist()) == fx.triangle_sets
        _check_listing_shape(dp, dc, lst)


def test_list_closed_forms():
    from math import comb
    # K_n: every 3-subset once
    for n in (3, 4, 7, 12):
        _, s, d = pins.complete(n)
        _, _, lst = _listing(n, s, d)
        sets = {tuple(sorted(r)) for r in lst.tolist()}
        assert len(lst) == len(sets) == comb(n, 3)
    # friendship F_k: k triangles, all through the centre
    for k in (1, 3, 6):
        n, s, d = pins.friendship(k)
        _, _, lst = _listing(n, s, d)
        assert len(lst) == k
        centre = np.bincount(lst.ravel(), minlength=n).argmax()
        assert all(centre in r for r in lst.tolist())
    # K_{a,b,c}: a*b*c triangles, one vertex from each part
    a, b, c = 2, 3, 4
    n, s, d = pins.complete_tripartite(a, b, c)
    _, _, lst = _listing(n, s, d)
    assert len(lst) == a * b * c
    part = np.array([0] * a + [1] * b + [2] * c)
    assert all(sorted(part[list(r)]) == [0, 1, 2] for r in lst.tolist())
    # triangle-free families list nothing
    for n, s, d in (pins.cycle(9), pins.petersen(), pins.complete_bipartite(4, 5)):
        assert len(_listing(n, s, d)[2]) == 0


@pytest.mark.parametrize("seed", range(3))
def test_list_counts_agree_with_trace(seed):
    """G(1024, 8192): the listing has trace(A^3)/6 rows and vertex x appears in diag(A^3)_x / 2."""
    s, d, n = graphgen.erdos_renyi(1024, 8192, seed)
    tt, tper = pins.trace_cube(n, s.numpy(), d.numpy())
    dp, dc, lst = _listing(n, s.numpy(), d.numpy())
    assert len(lst) == tt
    np.testing.assert_array_equal(np.bincount(lst.ravel(), minlength=n), tper)
    _check_listing_shape(dp, dc, lst)


# -- per-edge support -----------------------------------------------------------------------


def _support(n, s, d, order=oracle.ORDER_DEGREE):
    rp, col = oracle.clean(n, s, d)
    dp, dc = oracle.orient(rp, col, order)
    T, sup = oracle.edge_support(dp, dc)
    return dp, dc, T, sup


def _support_by_definition(n, s, d, dp, dc):
    """Support of each oriented edge {a, b}: common neighbours of a and b in the edge set."""
    nb = [set() for _ in range(n)]
    for a, b in pins.edge_set(s, d):
        nb[a].add(b)
        nb[b].add(a)
    return np.array([len(nb[u] & nb[int(v)]) for u in range(n) for v in dc[dp[u]:dp[u + 1]]],
                    dtype=np.uint32)


@pytest.mark.parametrize("seed", range(50))
def test_support_brute_force_random_tiny(seed):
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(1, 30))
    n, s, d = pins.random_simple(n, float(rng.choice([0.1, 0.3, 0.6, 1.0])), seed)
    bt, _ = pins.brute_force(n, s, d)
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        dp, dc, T, sup = _support(n, s, d, order)
        assert T == bt and int(sup.sum()) == 3 * bt
        np.testing.assert_array_equal(sup, _support_by_definition(n, s, d, dp, dc))


def test_support_closed_forms():
    # K_n: every edge lies in n - 2 triangles
    for n in (3, 5, 9):
        _, s, d = pins.complete(n)
        _, _, T, sup = _support(n, s, d)
        assert np.all(sup == n - 2) and sup.size == n * (n - 1) // 2
    # wheel with r >= 4 rim vertices: rim edges in 1 triangle, spokes in 2
    r = 7
    n, s, d = pins.wheel(r)
    dp, dc, T, sup = _support(n, s, d)
    for u in range(n):
        for k, v in enumerate(dc[dp[u]:dp[u + 1]]):
            assert sup[dp[u] + k] == (2 if 0 in (u, int(v)) else 1)
    # friendship F_k: every edge in exactly one triangle; triangle-free graphs: all zero
    n, s, d = pins.friendship(5)
    assert np.all(_support(n, s, d)[3] == 1)
    for n, s, d in (pins.cycle(8), pins.petersen(), pins.complete_bipartite(3, 4)):
        assert not _support(n, s, d)[3].any()


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_support_golden_fixtures(fx):
    """Support of each fixture edge = fixture triangles (hand-derived) containing both ends."""
    dp, dc, T, sup = _support(fx.n, fx.src, fx.dst)
    assert T == fx.triangles
    for u in range(fx.n):
        for k, v in enumerate(dc[dp[u]:dp[u + 1]]):
            want = sum(1 for t in fx.triangle_sets if u in t and int(v) in t)
            assert sup[dp[u] + k] == want


def test_support_config1_against_matrix_product():
    """G(1024, 8192): support of edge {a, b} = (A^2)[a, b], the common-neighbour count."""
    s, d, n = graphgen.erdos_renyi(1024, 8192, 1)
    a = np.zeros((n, n))
    a[s.numpy(), d.numpy()] = 1
    a[d.numpy(), s.numpy()] = 1
    np.fill_diagonal(a, 0)
    a2 = a @ a
    dp, dc, T, sup = _support(n, s.numpy(), d.numpy())
    rows = np.repeat(np.arange(n), np.diff(dp))
    np.testing.assert_array_equal(sup, a2[rows, dc].astype(np.uint32))


# -- the NE filter (k-core) ---------------------------------------------------------------


def _kcore_by_definition(n, s, d, k):
    """Repeatedly drop every vertex with fewer than k remaining neighbours (synchronous rounds)."""
    nb = [set() for _ in range(n)]
    for a, b in pins.edge_set(s, d):
        nb[a].add(b)
        nb[b].add(a)
    alive = set(range(n))
    while True:
        drop = {v for v in alive if len(nb[v] & alive) < k}
        if not drop:
            return np.array([1 if v in alive else 0 for v in range(n)], dtype=np.uint8)
        alive -= drop


@pytest.mark.parametrize("seed", range(40))
def test_kcore_by_definition_random_tiny(seed):
    rng = np.random.default_rng(6000 + seed)
    n = int(rng.integers(1, 40))
    n, s, d = pins.random_simple(n, float(rng.choice([0.03, 0.06, 0.1, 0.2, 0.5])), seed)
    rp, col = oracle.clean(n, s, d)
    for k in (1, 2, 3):
        np.testing.assert_array_equal(oracle.kcore(rp, col, k), _kcore_by_definition(n, s, d, k))


def test_kcore_closed_forms_and_count_preservation():
    def core(n, s, d, k=2):
        rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
        return oracle.kcore(rp, col, k)
    assert core(*pins.cycle(9)).all()              # 2-regular: all stay
    assert core(*pins.complete(6)).all()
    assert not core(*pins.star(7)).any()           # a tree peels away completely
    assert not core(8, list(range(7)), list(range(1, 8))).any()  # a path
    assert core(*pins.friendship(4)).all()         # centre degree 8, others degree 2
    # a triangle with a pendant path 2-3-4-5: only the triangle survives
    keep = core(6, [0, 1, 2, 2, 3, 4], [1, 2, 0, 3, 4, 5])
    np.testing.assert_array_equal(keep, [1, 1, 1, 0, 0, 0])
    # every triangle vertex survives the 2-core, so the count on the core is the count
    for seed in range(10):
        n, s, d = pins.random_simple(30, 0.08, seed)
        keep = core(n, s, d)
        e = [(a, b) for a, b in zip(s, d) if keep[a] and keep[b]]
        sub_s = [a for a, _ in e]
        sub_d = [b for _, b in e]
        assert oracle.triangles(n, np.array(sub_s, dtype=np.int32), np.array(sub_d, dtype=np.int32)) \
            == pins.brute_force(n, s, d)[0]


# -- 4-cliques ---------------------------------------------------------------------------------


def _k4_subsets(n, s, d):
    """Reference by enumeration of all 4-subsets (tiny n only)."""
    import itertools
    e = pins.edge_set(s, d)
    return sum(1 for q in itertools.combinations(range(n), 4)
               if all(frozenset(p) in e for p in itertools.combinations(q, 2)))


@pytest.mark.parametrize("seed", range(40))
def test_k4_brute_force_random_tiny(seed):
    rng = np.random.default_rng(8000 + seed)
    n = int(rng.integers(1, 22))
    n, s, d = pins.random_simple(n, float(rng.choice([0.2, 0.4, 0.6, 0.8, 1.0])), seed)
    want = _k4_subsets(n, s, d)
    assert pins.brute_force_k4(n, s, d) == want
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        assert oracle.k4(n, s, d, order=order) == want


def test_k4_closed_forms():
    from math import comb
    for n in (3, 4, 5, 8, 13):
        _, s, d = pins.complete(n)
        assert oracle.k4(n, s, d) == comb(n, 4)
    # complete tripartite graphs have no K4; complete 4-partite K_{a,b,c,d} has a*b*c*d
    n, s, d = pins.complete_tripartite(3, 4, 5)
    assert oracle.k4(n, s, d) == 0
    parts = [2, 3, 2, 4]
    off = np.cumsum([0] + parts)
    s4, d4 = [], []
    for p in range(4):
        for q in range(p + 1, 4):
            for i in range(off[p], off[p + 1]):
                for j in range(off[q], off[q + 1]):
                    s4.append(i)
                    d4.append(j)
    assert oracle.k4(int(off[-1]), s4, d4) == 2 * 3 * 2 * 4
    # wheels: W_3 = K4 has one, larger wheels none; friendship graphs none
    n, s, d = pins.wheel(3)
    assert oracle.k4(n, s, d) == 1
    for r in (4, 5, 9):
        n, s, d = pins.wheel(r)
        assert oracle.k4(n, s, d) == 0
    n, s, d = pins.friendship(5)
    assert oracle.k4(n, s, d) == 0


@pytest.mark.parametrize("seed", range(3))
def test_k4_small_rmat_against_edge_enumeration(seed):
    """R-MAT scale 9: against the independent edge-and-common-neighbour enumeration."""
    s, d, n = graphgen.rmat(9, 8, 300 + seed)
    want = pins.brute_force_k4(n, s.numpy(), d.numpy())
    assert want > 0
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        assert oracle.k4(n, s.numpy(), d.numpy(), order=order) == want


# -- diamonds (two triangles sharing an edge) -------------------------------------------------

def _diamond_maps(n, s, d):
    """The definition itself (Def. 2): injective maps of the query nodes (a, b, c, d) onto data
    vertices that send the five query edges a-b, a-c, b-c, b-d, c-d onto data edges, divided
    by the query's 4 automorphisms (swap a/d, swap b/c).  Tiny n only."""
    import itertools
    e = pins.edge_set(s, d)
    adj = lambda x, y: frozenset((x, y)) in e  # noqa: E731
    maps = sum(1 for a, b, c, dd in itertools.permutations(range(n), 4)
               if adj(a, b) and adj(a, c) and adj(b, c) and adj(b, dd) and adj(c, dd))
    assert maps % 4 == 0
    return maps // 4


def _diamond_subsets(n, s, d):
    """Per 4-subset: with e of its six pairs present it holds C(e, 5) diamonds (K4 minus any one
    edge is a diamond, and a diamond needs five edges).  Returns (diamonds, induced ones)."""
    import itertools
    from math import comb
    e = pins.edge_set(s, d)
    tot = ind = 0
    for q in itertools.combinations(range(n), 4):
        k = sum(1 for p in itertools.combinations(q, 2) if frozenset(p) in e)
        tot += comb(k, 5) if k >= 5 else 0
        ind += k == 5
    return tot, ind


@pytest.mark.parametrize("seed", range(30))
def test_diamonds_definition_random_tiny(seed):
    rng = np.random.default_rng(9100 + seed)
    n = int(rng.integers(1, 11))
    n, s, d = pins.random_simple(n, float(rng.choice([0.3, 0.5, 0.7, 0.9, 1.0])), seed)
    want = _diamond_maps(n, s, d)
    assert _diamond_subsets(n, s, d)[0] == want
    assert oracle.diamonds(n, s, d) == want
    n2, s2, d2 = pins.noisy(n, s, d, seed)  # duplicates, reversed pairs, self-loops
    assert oracle.diamonds(n2, s2, d2) == want


@pytest.mark.parametrize("seed", range(20))
def test_diamonds_are_induced_ones_plus_six_per_4_clique(seed):
    """Every K4 holds six diamonds, every other diamond is induced: pins the count against
    the 4-clique oracle and the induced count on random graphs up to 18 vertices."""
    rng = np.random.default_rng(9200 + seed)
    n = int(rng.integers(4, 19))
    n, s, d = pins.random_simple(n, float(rng.choice([0.3, 0.5, 0.7, 0.9])), seed)
    tot, ind = _diamond_subsets(n, s, d)
    assert oracle.diamonds(n, s, d) == tot == ind + 6 * oracle.k4(n, s, d)


def test_diamonds_closed_forms():
    from math import comb
    for n in range(0, 12):
        _, s, d = pins.complete(n)
        assert oracle.diamonds(n, s, d) == 6 * comb(n, 4)
    # wheels: W_3 = K4; from 4 rim vertices on, each spoke is the shared edge of one diamond
    n, s, d = pins.wheel(3)
    assert oracle.diamonds(n, s, d) == 6
    for r in range(4, 12):
        n, s, d = pins.wheel(r)
        assert oracle.diamonds(n, s, d) == r
    # book: the edge {0, 1} and k pages 2..k+1 adjacent to both
    for k in range(0, 9):
        s = [0] + [0] * k + [1] * k
        d = [1] + list(range(2, k + 2)) * 2
        assert oracle.diamonds(k + 2, s, d) == comb(k, 2)
    # complete tripartite: an edge between two parts has the third part as common neighbours
    for a, b, c in [(1, 1, 1), (2, 2, 2), (1, 2, 3), (3, 4, 5)]:
        n, s, d = pins.complete_tripartite(a, b, c)
        want = a * b * comb(c, 2) + a * c * comb(b, 2) + b * c * comb(a, 2)
        assert oracle.diamonds(n, s, d) == want
    # no two triangles share an edge
    for k in range(0, 6):
        n, s, d = pins.friendship(k)
        assert oracle.diamonds(n, s, d) == 0
    for n in range(3, 10):
        assert oracle.diamonds(*pins.cycle(n)) == 0
    for a, b in [(1, 1), (3, 3), (4, 7)]:
        assert oracle.diamonds(*pins.complete_bipartite(a, b)) == 0
    assert oracle.diamonds(*pins.petersen()) == 0
    assert oracle.diamonds(0, [], []) == 0


@pytest.mark.parametrize("seed", range(3))
def test_diamonds_small_rmat_against_edge_support(seed):
    """R-MAT scale 10: the diamonds sharing edge e are the pairs of triangles on e, so the count
    is the sum over edges of C(support, 2), with the support from the oriented-graph support
    oracle (another code path), in both orders; relabelling the vertices changes nothing."""
    s, d, n = graphgen.rmat(10, 8, 400 + seed)
    s, d = s.numpy(), d.numpy()
    want = oracle.diamonds(n, s, d)
    assert want > 0
    rp, col = oracle.clean(n, s, d)
    for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
        dp, dc = oracle.orient(rp, col, order)
        _, sup = oracle.edge_support(dp, dc)
        sup = sup.astype(np.int64)
        assert int((sup * (sup - 1) // 2).sum()) == want
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    assert oracle.diamonds(n, perm[s], perm[d]) == want
    # the bounded sample of the benchmark's baseline: all lower ends = the whole count
    assert oracle.count_diamonds(rp, col, sources=n) == want
    assert oracle.count_diamonds(rp, col, sources=0) == 0


# ---- labelled triangles ---------------------------------------------------------------

def _labels(n, k, seed):
    return np.random.default_rng(seed).integers(0, k, max(n, 1)).astype(np.int32)[:n]


@pytest.mark.parametrize("seed", range(12))
def test_labelled_brute_force_random_tiny(seed):
    """Every vertex triple checked for the three edges and the label multiset."""
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(3, 30))
    n, s, d = pins.random_simple(n, float(rng.choice([0.2, 0.5, 0.9])), seed)
    n, s, d = pins.noisy(n, s, d, seed)
    k = int(rng.integers(1, 4))
    lab = _labels(n, k, seed)
    tris = pins.brute_force_sets(n, s, d)
    for q in [(0, 0, 0), (0, 0, 1), (0, 1, 2), (1, 1, 2), (2, 1, 0), (0, 1, 1)]:
        want = sum(sorted(int(lab[x]) for x in t) == sorted(q) for t in tris)
        for order in (oracle.ORDER_DEGREE, oracle.ORDER_ID):
            assert oracle.labelled(n, s, d, lab, q, order=order) == want, (q, order)


def test_labelled_closed_forms():
    """K_n with label classes of sizes a, b, c: C(a,3) triangles labelled AAA, C(a,2) b AAB,
    a b c ABC; one label everywhere gives every triangle."""
    from math import comb
    a, b, c = 5, 4, 3
    n, s, d = pins.complete(a + b + c)
    lab = np.array([0] * a + [1] * b + [2] * c, dtype=np.int32)
    perm = np.random.default_rng(1).permutation(n)
    lab = lab[perm]  # labels need not follow the ids
    assert oracle.labelled(n, s, d, lab, (0, 0, 0)) == comb(a, 3)
    assert oracle.labelled(n, s, d, lab, (0, 1, 0)) == comb(a, 2) * b
    assert oracle.labelled(n, s, d, lab, (1, 2, 2)) == b * comb(c, 2)
    assert oracle.labelled(n, s, d, lab, (2, 1, 0)) == a * b * c
    assert oracle.labelled(n, s, d, lab, (3, 0, 0)) == 0
    assert oracle.labelled(n, s, d, np.zeros(n, np.int32), (0, 0, 0)) == comb(n, 3)
    # a wheel whose hub has its own label: every triangle is hub + two rim vertices
    k = 9
    s = [0] * k + list(range(1, k + 1))
    d = list(range(1, k + 1)) + [i % k + 1 for i in range(1, k + 1)]
    lab = np.array([5] + [7] * k, dtype=np.int32)
    assert oracle.labelled(k + 1, s, d, lab, (5, 7, 7)) == k
    assert oracle.labelled(k + 1, s, d, lab, (7, 7, 7)) == 0


def test_labelled_multisets_partition_the_triangles():
    """Summed over every label multiset, the labelled counts give the unlabelled total."""
    import itertools
    s, d, n = graphgen.rmat(9, 8, 5)
    s, d = s.numpy(), d.numpy()
    k = 3
    lab = _labels(n, k, 5)
    T = oracle.triangles(n, s, d)
    parts = sum(oracle.labelled(n, s, d, lab, q)
                for q in itertools.combinations_with_replacement(range(k), 3))
    assert parts == T > 0


# ---- directed triangles ---------------------------------------------------------------

# directed queries by their arcs on the nodes 0, 1, 2
_CYCLE = {(0, 1), (1, 2), (2, 0)}
_FFL = {(0, 1), (1, 2), (0, 2)}  # transitive (feed-forward) triangle
_ALL_ARCS = {(i, j) for i in range(3) for j in range(3) if i != j}


def _codes(arcs):
    """(p01, p02, p12): bit 1 = the lower node points to the higher, bit 2 = the reverse."""
    return tuple(int((i, j) in arcs) | 2 * int((j, i) in arcs) for i, j in ((0, 1), (0, 2), (1, 2)))


def _arcs(codes):
    out = set()
    for (i, j), c in zip(((0, 1), (0, 2), (1, 2)), codes):
        if c & 1:
            out.add((i, j))
        if c & 2:
            out.add((j, i))
    return out


def _perms3():
    import itertools
    return list(itertools.permutations(range(3)))


def _brute_directed(n, s, d, arcs_q, induced):
    """Every ordered triple of distinct vertices as the image of nodes 0, 1, 2, checked arc
    by arc; divided by the permutations of the query that keep its arcs."""
    A = {(int(a), int(b)) for a, b in zip(s, d) if a != b}
    emb = 0
    for x in range(n):
        for y in range(n):
            for z in range(n):
                if len({x, y, z}) < 3:
                    continue
                f = (x, y, z)
                ok = True
                for i in range(3):
                    for j in range(3):
                        if i == j:
                            continue
                        q, g = (i, j) in arcs_q, (f[i], f[j]) in A
                        if (q != g) if induced else (q and not g):
                            ok = False
                emb += ok
    aut = sum(all(((p[i], p[j]) in arcs_q) == ((i, j) in arcs_q)
                  for i in range(3) for j in range(3) if i != j) for p in _perms3())
    assert emb % aut == 0
    return emb // aut


def _random_digraph(n, p, seed):
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < p
    np.fill_diagonal(a, False)
    s, d = np.nonzero(a)
    # duplicates and self-loops, which add no arc
    extra = rng.integers(0, max(n, 1), size=(2, 3))
    s = np.concatenate([s, s[:2], extra[0], extra[0]])
    d = np.concatenate([d, d[:2], extra[0], extra[1]])
    return s.astype(np.int32), d.astype(np.int32)


@pytest.mark.parametrize("seed", range(10))
def test_directed_brute_force_random_tiny(seed):
    """All 27 directed triangle queries (every pair of query nodes joined by one arc either
    way or by both), induced and not, against brute force over ordered vertex triples."""
    import itertools
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(3, 11))
    s, d = _random_digraph(n, float(rng.choice([0.3, 0.5, 0.8])), seed)
    for codes in itertools.product((1, 2, 3), repeat=3):
        arcs_q = _arcs(codes)
        for induced in (False, True):
            want = _brute_directed(n, s, d, arcs_q, induced)
            order = oracle.ORDER_DEGREE if (seed + codes[0]) % 2 else oracle.ORDER_ID
            assert oracle.directed(n, s, d, codes, induced=induced, order=order) == want, \
                (codes, induced)


def test_directed_closed_forms():
    """Tournaments: a triangle is transitive iff one vertex points to both others, so there
    are sum_v C(out(v), 2) transitive triangles and C(n,3) minus that cyclic ones.  The
    complete symmetric digraph: every triangle holds 2 cycles and 6 transitive triangles,
    but as an induced subgraph is only the all-arcs query."""
    from math import comb
    for seed, n in ((1, 5), (2, 9), (3, 14)):
        rng = np.random.default_rng(seed)
        s, d = [], []
        for i in range(n):
            for j in range(i + 1, n):
                if rng.random() < 0.5:
                    s.append(i); d.append(j)
                else:
                    s.append(j); d.append(i)
        perm = rng.permutation(n)
        s, d = perm[np.array(s)], perm[np.array(d)]
        out = np.bincount(s, minlength=n)
        trans = sum(comb(int(o), 2) for o in out)
        for induced in (False, True):
            assert oracle.directed(n, s, d, _codes(_FFL), induced=induced) == trans
            assert oracle.directed(n, s, d, _codes(_CYCLE), induced=induced) == comb(n, 3) - trans
            assert oracle.directed(n, s, d, _codes(_ALL_ARCS), induced=induced) == 0
    n = 7
    s = np.array([i for i in range(n) for j in range(n) if i != j])
    d = np.array([j for i in range(n) for j in range(n) if i != j])
    assert oracle.directed(n, s, d, _codes(_CYCLE)) == 2 * comb(n, 3)
    assert oracle.directed(n, s, d, _codes(_FFL)) == 6 * comb(n, 3)
    assert oracle.directed(n, s, d, _codes(_ALL_ARCS)) == comb(n, 3)
    assert oracle.directed(n, s, d, _codes(_CYCLE), induced=True) == 0
    assert oracle.directed(n, s, d, _codes(_ALL_ARCS), induced=True) == comb(n, 3)
    # a directed cycle of length 3 and a longer one (no triangle)
    assert oracle.directed(3, [0, 1, 2], [1, 2, 0], _codes(_CYCLE)) == 1
    assert oracle.directed(3, [0, 1, 2], [1, 2, 0], _codes(_FFL)) == 0
    assert oracle.directed(5, [0, 1, 2, 3, 4], [1, 2, 3, 4, 0], _codes(_CYCLE)) == 0


def test_directed_triad_classes_partition_the_triangles():
    """Every triangle of the underlying graph is an induced match of exactly one of the 7
    classes of three-node digraphs with every pair joined; reversing every arc of the graph
    and of the query changes nothing."""
    import itertools
    s, d, n = graphgen.rmat(9, 8, 6)
    s, d = s.numpy(), d.numpy()
    # half the pairs also get the reverse arc
    both = np.arange(s.size) % 2 == 0
    s2 = np.concatenate([s, d[both]])
    d2 = np.concatenate([d, s[both]])
    T = oracle.triangles(n, s2, d2)
    classes = {}
    for codes in itertools.product((1, 2, 3), repeat=3):
        arcs = _arcs(codes)
        key = min(tuple(sorted((p[i], p[j]) for i, j in arcs)) for p in _perms3())
        classes.setdefault(key, codes)
    assert len(classes) == 7
    counts = {k: oracle.directed(n, s2, d2, c, induced=True) for k, c in classes.items()}
    assert sum(counts.values()) == T > 0
    assert min(counts.values()) > 0
    swap = {1: 2, 2: 1, 3: 3}
    for c in list(classes.values())[:4]:
        rc = tuple(swap[x] for x in c)
        for induced in (False, True):
            assert oracle.directed(n, d2, s2, rc, induced=induced) == \
                oracle.directed(n, s2, d2, c, induced=induced)
    # every arc reciprocal: the all-arcs query counts the undirected triangles
    s3, d3 = np.concatenate([s, d]), np.concatenate([d, s])
    assert oracle.directed(n, s3, d3, (3, 3, 3)) == oracle.triangles(n, s, d)


def test_directed_sources_sample():
    """The benchmark's bounded sample: the triangles whose DAG source lies below k; all
    sources give the whole count, none give 0, and the sample grows with k."""
    s, d, n = graphgen.rmat(8, 8, 3)
    s, d = s.numpy(), d.numpy()
    rp, col = oracle.clean(n, s, d)
    dp, dc = oracle.orient(rp, col)
    full = oracle.count_directed(dp, dc, s, d, _codes(_CYCLE))
    assert full > 0
    assert oracle.count_directed(dp, dc, s, d, _codes(_CYCLE), sources=n) == full
    assert oracle.count_directed(dp, dc, s, d, _codes(_CYCLE), sources=0) == 0
    parts = [oracle.count_directed(dp, dc, s, d, _codes(_CYCLE), sources=k)
             for k in range(0, n + 1, max(1, n // 8))]
    assert parts == sorted(parts)


# ---- edge-labelled triangles ---------------------------------------------------------

def _brute_edge_labelled(n, s, d, lab, q):
    """Every ordered triple of distinct vertices as the image of query nodes 0, 1, 2, with
    the label of each undirected edge the largest over its pairs; divided by the query's
    label-preserving node permutations."""
    import itertools
    L = {}
    for a, b, x in zip(s, d, lab):
        a, b, x = int(a), int(b), int(x)
        if a != b:
            key = (min(a, b), max(a, b))
            L[key] = max(L.get(key, x), x)
    qlab = {(0, 1): q[0], (0, 2): q[1], (1, 2): q[2]}
    emb = 0
    for f in itertools.permutations(range(n), 3):
        ok = True
        for (i, j), want in qlab.items():
            key = (min(f[i], f[j]), max(f[i], f[j]))
            if L.get(key) != want:
                ok = False
        emb += ok
    aut = sum(all(qlab[(min(p[i], p[j]), max(p[i], p[j]))] == qlab[(i, j)] for (i, j) in qlab)
              for p in itertools.permutations(range(3)))
    assert emb % aut == 0
    return emb // aut


@pytest.mark.parametrize("seed", range(8))
def test_edge_labelled_brute_force_random_tiny(seed):
    """All 27 queries over three edge labels, on random graphs whose pairs repeat with
    different labels (the largest counts), against brute force over ordered vertex triples."""
    import itertools
    rng = np.random.default_rng(1100 + seed)
    n = int(rng.integers(3, 12))
    n, s, d = pins.random_simple(n, float(rng.choice([0.3, 0.6, 0.9])), seed)
    n, s, d = pins.noisy(n, s, d, seed)
    s, d = np.asarray(s), np.asarray(d)
    lab = rng.integers(0, 3, size=s.size)
    for q in itertools.product(range(3), repeat=3):
        want = _brute_edge_labelled(n, s, d, lab, q)
        order = oracle.ORDER_DEGREE if (seed + q[0]) % 2 else oracle.ORDER_ID
        assert oracle.edge_labelled(n, s, d, lab, q, order=order) == want, q


def test_edge_labelled_closed_forms():
    """K_n with edge {i, j} labelled (i + j) mod 2: a triangle's three labels sum to an even
    number, so it is all-even (three vertices of one parity) or has two odd labels; one
    label everywhere gives every triangle."""
    from math import comb
    n = 11
    s = np.array([i for i in range(n) for j in range(i + 1, n)])
    d = np.array([j for i in range(n) for j in range(i + 1, n)])
    lab = (s + d) % 2
    e, o = (n + 1) // 2, n // 2
    assert oracle.edge_labelled(n, s, d, lab, (0, 0, 0)) == comb(e, 3) + comb(o, 3)
    assert oracle.edge_labelled(n, s, d, lab, (1, 0, 1)) == comb(e, 2) * o + comb(o, 2) * e
    assert oracle.edge_labelled(n, s, d, lab, (1, 1, 0)) == comb(e, 2) * o + comb(o, 2) * e
    assert oracle.edge_labelled(n, s, d, lab, (1, 1, 1)) == 0
    assert oracle.edge_labelled(n, s, d, lab, (0, 0, 1)) == 0
    assert oracle.edge_labelled(n, s, d, np.full(s.size, 2), (2, 2, 2)) == comb(n, 3)
    # a pair given twice with labels 0 and 3 carries 3
    assert oracle.edge_labelled(3, [0, 1, 2, 1], [1, 2, 0, 0], [0, 0, 0, 3], (0, 0, 3)) == 1
    assert oracle.edge_labelled(3, [0, 1, 2, 1], [1, 2, 0, 0], [0, 0, 0, 3], (0, 0, 0)) == 0


def test_edge_labelled_multisets_partition_the_triangles():
    """Summed over every multiset of three edge labels, the counts give the unlabelled
    total (a triangle matches exactly the query with its own label multiset, once)."""
    import itertools
    s, d, n = graphgen.rmat(9, 8, 7)
    s, d = s.numpy(), d.numpy()
    lab = np.random.default_rng(7).integers(0, 4, size=s.size)
    T = oracle.triangles(n, s, d)
    parts = sum(oracle.edge_labelled(n, s, d, lab, q)
                for q in itertools.combinations_with_replacement(range(4), 3))
    assert parts == T > 0


def test_edge_labelled_sources_sample():
    """The benchmark's bounded sample: all sources give the whole count, none give 0, and
    the sample grows with the bound."""
    s, d, n = graphgen.rmat(8, 8, 4)
    s, d = s.numpy(), d.numpy()
    lab = np.random.default_rng(4).integers(0, 2, size=s.size)
    rp, col = oracle.clean(n, s, d)
    dp, dc = oracle.orient(rp, col)
    full = oracle.count_edge_labelled(dp, dc, s, d, lab, (0, 1, 1))
    assert full > 0
    assert oracle.count_edge_labelled(dp, dc, s, d, lab, (0, 1, 1), sources=n) == full
    assert oracle.count_edge_labelled(dp, dc, s, d, lab, (0, 1, 1), sources=0) == 0
    parts = [oracle.count_edge_labelled(dp, dc, s, d, lab, (0, 1, 1), sources=k)
             for k in range(0, n + 1, max(1, n // 8))]
    assert parts == sorted(parts)
