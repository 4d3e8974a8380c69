"""GPU parity: every step of the HIP path against the CPU oracle, bit-exact.

Counts are integers, so the bar is equality: the cleaned CSR, the oriented DAG,
the total and every per-vertex count must match the oracle exactly.
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


def _gpu(tc, n, s, d, *, per_vertex=True, order=0, offset_bytes=4, tune=None):
    res = tc.triangle_count(_dev(s), _dev(d), n, per_vertex=per_vertex, order=order,
                            offset_bytes=offset_bytes, tune=tune)
    pv = res.per_vertex.cpu().numpy().astype(np.uint64) if per_vertex else None
    return res, pv


def _oracle(n, s, d, order=0):
    return oracle.triangles(n, np.asarray(s), np.asarray(d), per_vertex=True, order=order)


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_golden_fixtures(tc, fx):
    _say("golden", fx.name)
    for order in (tc.TC_ORDER_DEGREE, tc.TC_ORDER_ID):
        for ob in (4, 8):
            res, pv = _gpu(tc, fx.n, fx.src, fx.dst, order=order, offset_bytes=ob)
            assert res.total == fx.triangles
            np.testing.assert_array_equal(pv, fx.per_vertex)


@pytest.mark.parametrize("case", pins.closed_form_cases(), ids=lambda c: c[0])
def test_closed_forms(tc, case):
    name, (n, s, d), T, t = case
    _say("closed form", name)
    res, pv = _gpu(tc, n, s, d)
    assert res.total == T
    assert int(pv.sum()) == 3 * T
    if t is not None:
        np.testing.assert_array_equal(pv, t)
    res2, _ = _gpu(tc, n, s, d, per_vertex=False, order=tc.TC_ORDER_ID)
    assert res2.total == T


def test_random_tiny_against_oracle(tc):
    for seed in range(60):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 48))
        n, s, d = pins.random_simple(n, float(rng.choice([0.1, 0.3, 0.6, 1.0])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        _say("tiny seed", seed, "n", n, "pairs", len(s))
        T, t = _oracle(n, s, d)
        for order in (0, 1):
            res, pv = _gpu(tc, n, s, d, order=order, offset_bytes=4 + 4 * (seed % 2))
            assert res.total == T
            np.testing.assert_array_equal(pv, t)


def _csr_parity(tc, n, s, d, offset_bytes):
    p = tc.Pipeline(n, len(s), offset_bytes=offset_bytes)
    p.build(_dev(s), _dev(d))
    torch.cuda.synchronize()
    nnz = int(p.nnz.item())
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    assert nnz == rp[-1]
    np.testing.assert_array_equal(p.row_ptr.cpu().numpy().astype(np.int64), rp)
    np.testing.assert_array_equal(p.col[:nnz].cpu().numpy(), col)
    for order in (0, 1):
        p.order = order
        p.orient()
        torch.cuda.synchronize()
        m = int(p.m.item())
        dp, dc = oracle.orient(rp, col, order)
        assert m == dp[-1]
        np.testing.assert_array_equal(p.dag_ptr.cpu().numpy().astype(np.int64), dp)
        np.testing.assert_array_equal(p.dag_col[:m].cpu().numpy(), dc)


@pytest.mark.parametrize("n,pairs,seed", [(1, 5, 0), (2, 9, 1), (7, 40, 2), (100, 3000, 3),
                                          (1000, 50000, 4), (4097, 70000, 5), (65536, 300000, 6),
                                          (70001, 900000, 7)])
def test_build_and_orient_bit_exact(tc, n, pairs, seed):
    """Uniform random pairs: heavy duplication, both directions, self-loops."""
    _say("build/orient", n, pairs)
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, pairs)
    d = rng.integers(0, n, pairs)
    _csr_parity(tc, n, s, d, 4 + 4 * (seed % 2))


@pytest.mark.parametrize("scale,ef,seed", [(10, 16, 1), (14, 16, 2), (16, 8, 3)])
def test_rmat_build_orient_count(tc, scale, ef, seed):
    """Skewed R-MAT: hub rows (long-row path), workgroup-mode sources, several radix passes."""
    s, d, n = graphgen.rmat(scale, ef, seed)
    s, d = s.numpy(), d.numpy()
    _say("rmat", scale, ef)
    _csr_parity(tc, n, s, d, 4)
    T, t = _oracle(n, s, d)
    for order, ob in [(0, 4), (0, 8), (1, 4)]:
        res, pv = _gpu(tc, n, s, d, order=order, offset_bytes=ob)
        assert res.total == T
        np.testing.assert_array_equal(pv, t)


def test_config1_all_seeds(tc):
    """G(n=1024, m=8192), seeds 0-9, against the stored oracle counts."""
    import json
    import os
    with open(os.path.join(goldens.GOLDEN_DIR, "er1024_8192.json")) as f:
        data = json.load(f)
    for seed in range(10):
        s, d, n = graphgen.erdos_renyi(1024, 8192, seed)
        g = data["graphs"][str(seed)]
        res, pv = _gpu(tc, n, s.numpy(), d.numpy())
        assert res.total == g["triangles"] and res.m == 8192
        np.testing.assert_array_equal(pv, np.array(g["per_vertex"], dtype=np.uint64))


def _hub_graph(n_leaves, extra, seed):
    """Vertex 0 adjacent to every other vertex plus random edges among the others:
    under id order N+(0) holds every vertex, far beyond one LDS table slice."""
    rng = np.random.default_rng(seed)
    n = n_leaves + 1
    s = [0] * n_leaves + list(rng.integers(1, n, extra))
    d = list(range(1, n)) + list(rng.integers(1, n, extra))
    return n, np.array(s), np.array(d)


def test_hub_beyond_one_table_slice(tc):
    """Under id order N+(0) holds 5000 ids: beyond four table slices, so the source binary
    searches its row in memory; with both offset widths."""
    n, s, d = _hub_graph(5000, 40000, 11)
    _say("hub", n)
    T, t = _oracle(n, s, d)
    for order in (0, 1):
        for ob in (4, 8):
            res, pv = _gpu(tc, n, s, d, order=order, offset_bytes=ob)
            assert res.total == T
            np.testing.assert_array_equal(pv, t)


def test_dense_clique_all_source_classes(tc):
    """K_300 under id order gives sources of every out-degree 0..299."""
    n, s, d = pins.complete(300)
    res, pv = _gpu(tc, n, s, d, order=1)
    assert res.total == 300 * 299 * 298 // 6
    assert np.all(pv == 299 * 298 // 2)


def test_empty_and_degenerate(tc):
    for n, s, d in [(0, [], []), (1, [], []), (5, [], []), (5, [2, 2, 3], [2, 2, 3]),
                    (3, [0, 1, 2], [1, 2, 0])]:
        T, t = _oracle(n, s, d)
        if n == 0:
            res = tc.triangle_count(_dev(s), _dev(d), n)
            assert res.total == 0 and res.nnz == 0
            continue
        res, pv = _gpu(tc, n, s, d)
        assert res.total == T
        np.testing.assert_array_equal(pv, t)


def test_device_errors(tc):
    with pytest.raises(tc.TcError) as e:
        tc.triangle_count(_dev([0, 1, 5]), _dev([1, 2, 0]), 4)
    assert e.value.status == 2  # TC_ERR_ID_OUT_OF_RANGE
    with pytest.raises(tc.TcError) as e:
        tc.triangle_count(_dev([0, -1]), _dev([1, 2]), 4)
    assert e.value.status == 2
    # an orientation output that is too small
    p = tc.Pipeline(10, 20)
    s, d = pins.complete(5)[1:]
    p.build(_dev(s), _dev(d))
    small = torch.empty(3, dtype=torch.int32, device="cuda")
    from paper_1909_02127_amd import _lib
    _lib.tc_orient(10, p.row_ptr, p.col, 0, p.dag_ptr, small, p.m, p.ws_orient)
    torch.cuda.synchronize()
    assert int(p.m.item()) == -3
    assert int(p.dag_ptr.abs().sum().item()) == 0
    # a symmetric output that is too small
    nnz = torch.zeros(1, dtype=torch.int64, device="cuda")
    rp = torch.empty(11, dtype=torch.int32, device="cuda")
    col = torch.empty(5, dtype=torch.int32, device="cuda")
    _lib.tc_build_csr(10, _dev(s), _dev(d), rp, col, nnz, p.ws_build)
    torch.cuda.synchronize()
    assert int(nnz.item()) == -3 and int(rp.abs().sum().item()) == 0
    # a workspace that is too small is refused on the host
    with pytest.raises(tc.TcError) as e:
        _lib.tc_count(10, p.dag_ptr, p.dag_col, p.total, p.ws_count[:16])
    assert e.value.status == 4


def test_repeat_is_deterministic(tc):
    s, d, n = graphgen.rmat(13, 16, 4)
    p = tc.Pipeline(n, s.numel())
    src, dst = s.cuda(), d.cuda()
    first = None
    for _ in range(5):
        p.enqueue(src, dst, per_vertex=True)
        r = p.result(per_vertex=True)
        if first is None:
            first = r
        assert r.total == first.total
        assert torch.equal(r.per_vertex, first.per_vertex)


def test_generator_device_path_matches_cpu(tc):
    s1, d1, _ = graphgen.rmat(12, 8, 21)
    s2, d2, _ = graphgen.rmat(12, 8, 21, device="cuda")
    assert torch.equal(s1, s2.cpu()) and torch.equal(d1, d2.cpu())
    e1 = graphgen.erdos_renyi(5000, 30000, 3)
    e2 = graphgen.erdos_renyi(5000, 30000, 3, device="cuda")
    assert torch.equal(e1[0], e2[0].cpu()) and torch.equal(e1[1], e2[1].cpu())


def test_rmat_scale20_full_parity(tc):
    """The benchmark graph itself (R-MAT scale 20, edge factor 16) in the benchmark's launch
    configuration: total and all per-vertex counts against the oracle."""
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    _say("scale 20: gpu")
    p = tc.Pipeline(n, s.numel(), offset_bytes=4)
    p.enqueue(s, d, per_vertex=True)
    r = p.result(per_vertex=True)
    p.enqueue(s, d, per_vertex=False)
    r2 = p.result()
    assert r2.total == r.total
    _say("scale 20: oracle", r.total, r.m)
    hs, hd = s.cpu().numpy(), d.cpu().numpy()
    T, t = oracle.triangles(n, hs, hd, per_vertex=True)
    assert r.total == T
    np.testing.assert_array_equal(r.per_vertex.cpu().numpy().astype(np.uint64), t)
    rng = np.random.default_rng(0)
    for v in rng.choice(np.flatnonzero(t), 3, replace=False):
        assert oracle.vertex_triangles(n, hs, hd, int(v)) == int(t[v])


@pytest.mark.slow
def test_rmat_scale24_full_parity(tc):
    """R-MAT scale 24, edge factor 16, seed 24 with int64 offsets, in the benchmark's launch
    configuration: T > 2^32 and every t(v).  The oracle's counts are stored by
    tests/golden/make_rmat_s24.py (minutes of CPU): the total, sum(t) = 3T, t(v) of 576
    vertices (the 64 largest and 512 random ones) and the SHA-256 of the whole t array, which
    checks every t(v) at once.  Two t(v) are also recomputed here from the raw pairs."""
    import hashlib
    import json
    import os
    with open(os.path.join(goldens.GOLDEN_DIR, "rmat_s24_ef16_seed24.json")) as f:
        g = json.load(f)
    s, d, n = graphgen.rmat(24, 16, 24, device="cuda")
    _say("scale 24: gpu", n, s.numel())
    p = tc.Pipeline(n, s.numel(), offset_bytes=8)
    p.enqueue(s, d, per_vertex=True)
    r = p.result(per_vertex=True)
    assert (r.nnz, r.m) == (g["nnz"], g["m"])
    assert r.total == g["triangles"] and r.total > 2**32
    p.count()
    assert p.result().total == r.total
    t = np.ascontiguousarray(r.per_vertex.cpu().numpy().view(np.uint64), dtype="<u8")
    del r
    _say("scale 24: T", g["triangles"], "checking t")
    assert int(t.sum(dtype=np.uint64)) == g["sum_t"] == 3 * g["triangles"]
    for v, c in g["t_sample"].items():
        assert int(t[int(v)]) == c, v
    assert hashlib.sha256(t.tobytes()).hexdigest() == g["t_sha256"]
    hs, hd = s.cpu().numpy(), d.cpu().numpy()
    del p
    # vertices whose t is near 1e5 and near 1e3 (the definition scans all pairs once each)
    for want in (10**5, 10**3):
        v = int(min(g["t_sample"], key=lambda x: abs(g["t_sample"][x] - want)))
        assert oracle.vertex_triangles(n, hs, hd, v) == int(t[v]), v


@pytest.mark.parametrize("kicks", [-1, 1, 2])
def test_probe_fallback_modes(tc, kicks):
    """Capping cuckoo placements (tc_tune.max_kicks) pushes keys into the stash (1-2
    placements, small tables) and past it into the sorted binary-search fallback (-1: no
    placement, tables over 32 keys); counts must not change."""
    tune = {"max_kicks": kicks}
    cases = [pins.complete(40), pins.wheel(30), _hub_graph(1500, 9000, 3)]
    s, d, n = graphgen.rmat(12, 16, 8)
    cases.append((n, s.numpy(), d.numpy()))
    for n, s, d in cases:
        T, t = _oracle(n, s, d)
        for order in (0, 1):
            res, pv = _gpu(tc, n, s, d, order=order, tune=tune)
            assert res.total == T
            np.testing.assert_array_equal(pv, t)


def test_ids_above_2_24(tc):
    """Vertex ids beyond 2^24 take the folded (wide) hash; counts must not change."""
    rng = np.random.default_rng(24)
    base = (1 << 24) + 777
    n = base + 6000
    k = 60000
    s = rng.integers(base, n, k)
    d = rng.integers(base, n, k)
    # some edges between high and low ids, and a dense block of consecutive high ids
    s = np.concatenate([s, rng.integers(0, 5000, 3000), np.repeat(np.arange(base, base + 40), 40)])
    d = np.concatenate([d, rng.integers(base, n, 3000), np.tile(np.arange(base, base + 40), 40)])
    T, t = _oracle(n, s, d)
    for order in (0, 1):
        res, pv = _gpu(tc, n, s, d, order=order)
        assert res.total == T
        np.testing.assert_array_equal(pv, t)


def test_wave_workgroup_split_thresholds(tc):
    """Dense graphs put many sources at d+ in (64, 96]: every split between the one-wave
    and the workgroup path (tc_tune.small_max) gives the oracle's total and t(v)."""
    from paper_1909_02127_amd import _lib
    for n, m, seed in [(400, 30000, 7), (1500, 60000, 8)]:
        s, d, n = graphgen.erdos_renyi(n, m, seed)
        s, d = s.numpy(), d.numpy()
        T, t = _oracle(n, s, d)
        p = tc.Pipeline(n, len(s))
        p.build(_dev(s), _dev(d))
        p.orient()
        dplus = np.diff(p.dag_ptr.cpu().numpy())
        _say("split thresholds n", n, "sources with 64 < d+ <= 96:", int(((dplus > 64) & (dplus <= 96)).sum()))
        assert ((dplus > 64) & (dplus <= 96)).sum() > 0
        total = torch.zeros(1, dtype=torch.int64, device="cuda")
        pv = torch.zeros(n, dtype=torch.int64, device="cuda")
        ws = torch.empty(_lib.tc_count_per_vertex_workspace(n), dtype=torch.uint8, device="cuda")
        for sm in (0, 1, 64, 65, 80, 95, 96):
            tune = {"small_max": sm}
            _lib.tc_count_per_vertex(n, p.dag_ptr, p.dag_col, pv, total, ws, tune=tune)
            torch.cuda.synchronize()
            assert int(total.item()) == T, sm
            np.testing.assert_array_equal(pv.cpu().numpy().astype(np.uint64), t)
            _lib.tc_count(n, p.dag_ptr, p.dag_col, total, ws, tune=tune)
            torch.cuda.synchronize()
            assert int(total.item()) == T, sm
        with pytest.raises(_lib.TcError):
            _lib.tc_count(n, p.dag_ptr, p.dag_col, total, ws, tune={"small_max": 97})


@pytest.mark.parametrize("split_log2", [1, 6, 10, -1])
def test_equal_work_quanta(tc, split_log2):
    """Workgroup-mode sources whose work w(u) (wedges) exceeds 2^split_log2 are cut into
    parts that any workgroup may claim (tc_tune.split_log2).  Small quanta split almost
    every such source, in both orders and with per-vertex counts; counts must not change.
    Splitting 1 ("2 wedges per part") also runs into the 1024-part cap and, with several
    thousand heavy sources, into the full split table."""
    tune = {"split_log2": split_log2, "small_max": 16}
    cases = [pins.complete(60), _hub_graph(3000, 20000, 5)]
    s, d, n = graphgen.rmat(13, 16, 9)
    cases.append((n, s.numpy(), d.numpy()))
    s, d, n = graphgen.erdos_renyi(20000, 400000, 3)
    cases.append((n, s.numpy(), d.numpy()))
    for n, s, d in cases:
        _say("quanta", split_log2, "n", n, "pairs", len(s))
        T, t = _oracle(n, s, d)
        for order in (0, 1):
            res, pv = _gpu(tc, n, s, d, order=order, tune=tune)
            assert res.total == T
            np.testing.assert_array_equal(pv, t)
            res2, _ = _gpu(tc, n, s, d, order=order, tune=tune, per_vertex=False,
                           offset_bytes=8)
            assert res2.total == T
