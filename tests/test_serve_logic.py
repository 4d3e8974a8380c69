"""Serving-loop scheduling on the CPU: admission by footprint, FIFO order, lanes,
no starvation and rejection, with a fake executor whose answers come from the oracle."""
import numpy as np

import graphgen
import oracle
from paper_1909_02127_amd.serve import Engine, Request, footprint_bytes


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4  # time advances with every look at the clock
        return self.t


class FakeExecutor:
    """Completes a batch a fixed number of polls after launch; counts via the oracle."""

    def __init__(self, polls=3):
        self.polls = polls
        self.launched = []

    def launch(self, reqs):
        self.launched.append([r.rid for r in reqs])
        return {"reqs": reqs, "left": self.polls}

    def ready(self, h):
        h["left"] -= 1
        return h["left"] <= 0

    def collect(self, h):
        tot, pv = [], []
        for r in h["reqs"]:
            t, p = oracle.triangles(r.n, np.asarray(r.src), np.asarray(r.dst), per_vertex=True)
            tot.append(t)
            pv.append(p)
        return tot, pv


def _requests(k, large_every=0):
    out = []
    for i in range(k):
        if large_every and i % large_every == 0:
            s, d, n = graphgen.rmat(10, 16, 100 + i)
        else:
            s, d, n = graphgen.erdos_renyi(200, 800, i)
        out.append(Request(i, n, s.numpy(), d.numpy(), arrival=i * 1e-4))
    return out


def test_all_complete_with_correct_counts_and_budget_respected():
    reqs = _requests(40, large_every=9)
    budget = 3 * max(footprint_bytes(r.n, r.num_pairs) for r in reqs)
    eng = Engine(FakeExecutor(), budget_bytes=budget, max_inflight=3, max_batch=8,
                 large_pairs=10_000, clock=FakeClock())
    st = eng.run(reqs, idle_sleep=0)
    assert st.completed == 40 and st.rejected == 0
    assert st.max_in_use <= budget
    assert st.max_inflight_batches <= 3
    for r in reqs:
        t, p = oracle.triangles(r.n, r.src, r.dst, per_vertex=True)
        assert r.total == t
        np.testing.assert_array_equal(r.per_vertex, p)
        assert r.done >= r.arrival
    # large requests ran alone in their own batches
    large = {r.rid for r in reqs if r.num_pairs >= 10_000}
    for b in eng.ex.launched:
        if large & set(b):
            assert len(b) == 1


def test_oversized_request_is_rejected_not_blocking():
    reqs = _requests(6)
    big = Request(99, 10**6, np.zeros(10**6, np.int32), np.ones(10**6, np.int32), arrival=0.0)
    budget = 4 * footprint_bytes(reqs[0].n, reqs[0].num_pairs)
    eng = Engine(FakeExecutor(), budget_bytes=budget, clock=FakeClock())
    st = eng.run([big] + reqs, idle_sleep=0)
    assert st.rejected == 1 and big.error and big.total is None
    assert st.completed == 6


def test_fifo_admission_under_a_tight_budget():
    reqs = _requests(12)
    budget = footprint_bytes(reqs[0].n, reqs[0].num_pairs) + 1  # one request at a time
    eng = Engine(FakeExecutor(polls=2), budget_bytes=budget, clock=FakeClock())
    eng.run(reqs, idle_sleep=0)
    order = [rid for b in eng.ex.launched for rid in b]
    assert order == sorted(order)
    assert all(len(b) == 1 for b in eng.ex.launched)


def test_summary_percentiles():
    reqs = _requests(30)
    eng = Engine(FakeExecutor(), budget_bytes=1 << 40, clock=FakeClock())
    st = eng.run(reqs, idle_sleep=0)
    s = st.summary()
    assert s["completed"] == 30 and s["p50_ms"] <= s["p99_ms"]
    assert s["graphs_per_s"] > 0
