"""The serving loop on the GPU: every request's counts are the same alone and in the mix
(tolerance 0), batches overlap on the device, and the memory budget holds."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_02127_amd as tc
    return tc


def _pool():
    graphs = []
    for g in graphgen.batch_suite_spec(40, seed=12, log2_min=6, log2_max=12):
        graphs.append(graphgen.batch_graph(g))
    graphs.append(graphgen.rmat(15, 16, 5))        # a large request: its own lane
    graphs.append(graphgen.erdos_renyi(3, 0, 1))   # no edges
    return graphs


def test_alone_equals_in_the_mix(tc):
    from paper_1909_02127_amd.serve import DeviceExecutor, Engine, Request
    pool = _pool()
    alone = []
    for s, d, n in pool:
        r = tc.triangle_count(s.cuda(), d.cuda(), n, per_vertex=True)
        alone.append((r.total, r.per_vertex.cpu().numpy().astype(np.uint64)))
    rng = np.random.default_rng(3)
    reqs = []
    t = 0.0
    for i in range(3 * len(pool)):
        k = i % len(pool)
        s, d, n = pool[k]
        t += float(rng.exponential(1 / 4000.0))
        reqs.append(Request(i, n, s.pin_memory(), d.pin_memory(), arrival=t))
    budget = 1 << 30
    eng = Engine(DeviceExecutor(), budget_bytes=budget, max_inflight=3, max_batch=16,
                 large_pairs=200_000)
    st = eng.run(reqs)
    assert st.completed == len(reqs) and st.rejected == 0
    assert st.max_in_use <= budget
    assert st.batches > 3
    for i, r in enumerate(reqs):
        t_alone, pv_alone = alone[i % len(pool)]
        assert r.total == t_alone, i
        np.testing.assert_array_equal(r.per_vertex, pv_alone)
    for k in (0, 7, len(pool) - 2):
        s, d, n = pool[k]
        assert oracle.triangles(n, s.numpy(), d.numpy()) == alone[k][0]


def test_budget_smaller_than_the_mix(tc):
    """A budget of about two requests forces admission to wait; nothing is lost."""
    from paper_1909_02127_amd.serve import DeviceExecutor, Engine, Request, footprint_bytes
    pool = _pool()[:12]
    reqs = [Request(i, n, s.pin_memory(), d.pin_memory(), arrival=0.0)
            for i, (s, d, n) in enumerate(pool)]
    budget = 2 * max(footprint_bytes(r.n, r.num_pairs) for r in reqs)
    eng = Engine(DeviceExecutor(), budget_bytes=budget, max_inflight=3)
    st = eng.run(reqs)
    assert st.completed == len(reqs)
    assert st.max_in_use <= budget
    for r, (s, d, n) in zip(reqs, pool):
        assert r.total == oracle.triangles(n, s.numpy(), d.numpy())
