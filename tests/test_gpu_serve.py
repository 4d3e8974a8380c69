"""The serving loop on the GPU: every request's total and per-vertex counts equal the oracle's
and the same graph's counts alone (tolerance 0), batches on several lanes are in flight
together, large requests (R-MAT scale 18) take the large lane, and bad requests are
rejected without stopping the loop."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import graphgen
import oracle

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


@pytest.fixture(scope="module")
def pool():
    graphs = []
    for g in graphgen.batch_suite_spec(40, seed=12, log2_min=6, log2_max=12):
        graphs.append(graphgen.batch_graph(g))
    graphs.append(graphgen.rmat(15, 16, 5))        # large: over the small lanes' 400K pairs
    graphs.append(graphgen.rmat(18, 16, 6))        # large: 4.2M pairs
    graphs.append(graphgen.erdos_renyi(3, 0, 1))   # no edges
    want = []
    for s, d, n in graphs:
        want.append(oracle.triangles(n, s.numpy(), d.numpy(), per_vertex=True))
    return graphs, want


def _lanes(tc, small=3):
    from paper_1909_02127_amd import _lib
    from paper_1909_02127_amd.serve import plan_lanes
    return plan_lanes(_lib, 8 << 30, small_lanes=small, small_pairs=400_000,
                      small_vertices=200_000, small_graphs=16, large_lanes=1,
                      large_pairs=5_000_000, large_vertices=1 << 18)


def test_every_request_equals_the_oracle_and_alone(tc, pool):
    from paper_1909_02127_amd.serve import DeviceExecutor, Engine, Request
    graphs, want = pool
    alone = []
    for s, d, n in graphs:
        r = tc.triangle_count(s.cuda(), d.cuda(), n, per_vertex=True)
        alone.append((r.total, r.per_vertex.cpu().numpy().astype(np.uint64)))
    for (T, t), (Ta, ta) in zip(want, alone):
        assert T == Ta
        np.testing.assert_array_equal(t, ta)
    rng = np.random.default_rng(3)
    reqs = []
    t = 0.0
    for i in range(3 * len(graphs)):
        k = i % len(graphs)
        s, d, n = graphs[k]
        t += float(rng.exponential(1 / 4000.0))
        # half the requests hand over pinned tensors, half numpy arrays (staged)
        src, dst = (s.pin_memory(), d.pin_memory()) if i % 2 else (s.numpy(), d.numpy())
        reqs.append(Request(i, n, src, dst, arrival=t))
    lanes = _lanes(tc)
    ex = DeviceExecutor(lanes)
    eng = Engine(ex)
    st = eng.run(reqs)
    _say("serve:", st.summary())
    assert st.completed == len(reqs) and st.rejected == 0 and st.failed == 0
    assert st.max_inflight_batches >= 2
    assert st.large_batches >= 6  # the two large graphs, three times each
    assert st.max_in_use <= sum(ln.bytes for ln in lanes)
    for i, r in enumerate(reqs):
        T, tv = want[i % len(graphs)]
        assert r.total == T, i
        np.testing.assert_array_equal(r.per_vertex, tv)


def test_one_request_per_lane_and_rejections(tc, pool):
    """Lanes that hold one graph each force one request per batch; an invalid request and
    one larger than every lane are rejected and the others still complete."""
    from paper_1909_02127_amd import _lib
    from paper_1909_02127_amd.serve import DeviceExecutor, Engine, Lane, Request, lane_bytes
    graphs, want = pool
    small = graphs[:12]
    lanes = [Lane(0, False, 400_000, 200_000, 1, lane_bytes(_lib, 400_000, 200_000, 1))]
    reqs = [Request(i, n, s.numpy(), d.numpy(), arrival=0.0)
            for i, (s, d, n) in enumerate(small)]
    bad = Request(100, 5, np.array([0, 5], np.int32), np.array([1, 2], np.int32))
    big = Request(101, graphs[-2][2], graphs[-2][0].numpy(), graphs[-2][1].numpy())
    eng = Engine(DeviceExecutor(lanes))
    st = eng.run([bad, big] + reqs)
    assert st.completed == len(reqs) and st.rejected == 2 and st.batches == len(reqs)
    assert bad.error and big.error and bad.total is None and big.total is None
    for r, (T, tv) in zip(reqs, want[:12]):
        assert r.total == T
        np.testing.assert_array_equal(r.per_vertex, tv)


def test_pack_pairs_maps_out_of_range_ids_to_an_error(tc):
    """A local id beyond its graph's range becomes -1 in the union, which tc_build_csr
    reports as TC_ERR_ID_OUT_OF_RANGE (the device-side guard behind host validation)."""
    from paper_1909_02127_amd import _lib
    src = torch.tensor([0, 1, 0, 2], dtype=torch.int32, device="cuda")
    dst = torch.tensor([1, 2, 1, 3], dtype=torch.int32, device="cuda")
    pair_off = torch.tensor([0, 2, 4], dtype=torch.int64, device="cuda")
    vtx_off = torch.tensor([0, 3, 6], dtype=torch.int64, device="cuda")
    _lib.tc_pack_pairs(pair_off, vtx_off, src, dst)
    torch.cuda.synchronize()
    assert src.tolist() == [0, 1, 3, 5] and dst.tolist() == [1, 2, 4, -1]
