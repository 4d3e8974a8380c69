"""Serving-loop scheduling on the CPU: validation and routing by size, per-lane capacity,
FIFO order within a queue, small requests never behind large ones, error isolation and
rejection, with a fake executor whose answers come from the oracle."""
import numpy as np
import pytest

import graphgen
import oracle
from paper_1909_02127_amd.serve import Engine, Lane, Request, validate


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4  # time advances with every look at the clock
        return self.t


class FakeExecutor:
    """Completes a batch a fixed number of polls after launch; counts via the oracle.
    A batch that holds a request with `fail` set reports a device error."""

    def __init__(self, lanes, polls=3):
        self.lanes = lanes
        self.polls = polls
        self.launched = []  # (lane, [rid, ...])

    def launch(self, lane, reqs):
        assert self.lanes[lane].fits(sum(r.num_pairs for r in reqs), sum(r.n for r in reqs),
                                     len(reqs))
        self.launched.append((lane, [r.rid for r in reqs]))
        return {"reqs": reqs, "left": self.polls}

    def ready(self, h):
        h["left"] -= 1
        return h["left"] <= 0

    def collect(self, h):
        if any(getattr(r, "fail", False) for r in h["reqs"]):
            return None, None, "tc_build_csr: TC_ERR_ID_OUT_OF_RANGE"
        tot, pv = [], []
        for r in h["reqs"]:
            t, p = oracle.triangles(r.n, np.asarray(r.src), np.asarray(r.dst), per_vertex=True)
            tot.append(t)
            pv.append(p)
        return tot, pv, None


def _lanes(small=3, large=1, small_pairs=4000, large_pairs=100_000, graphs=8):
    out = []
    for _ in range(large):
        out.append(Lane(len(out), True, large_pairs, 1 << 16, 1, 10 * large_pairs))
    for _ in range(small):
        out.append(Lane(len(out), False, small_pairs, small_pairs, graphs, 10 * small_pairs))
    return out


def _requests(k, large_every=0):
    out = []
    for i in range(k):
        if large_every and i % large_every == 0:
            s, d, n = graphgen.rmat(10, 16, 100 + i)
        else:
            s, d, n = graphgen.erdos_renyi(200, 800, i)
        out.append(Request(i, n, s.numpy(), d.numpy(), arrival=i * 1e-4))
    return out


def test_all_complete_with_correct_counts_within_lane_capacity():
    reqs = _requests(40, large_every=9)
    ex = FakeExecutor(_lanes())
    eng = Engine(ex, clock=FakeClock())
    st = eng.run(reqs, idle_sleep=0)
    assert st.completed == 40 and st.rejected == 0 and st.failed == 0
    assert st.max_inflight_batches >= 2
    assert st.max_in_use <= sum(ln.bytes for ln in ex.lanes)
    for r in reqs:
        t, p = oracle.triangles(r.n, r.src, r.dst, per_vertex=True)
        assert r.total == t
        np.testing.assert_array_equal(r.per_vertex, p)
        assert r.done >= r.arrival
    large = {r.rid for r in reqs if r.num_pairs > 4000}
    assert large
    for lane, rids in ex.launched:
        if large & set(rids):
            assert ex.lanes[lane].large and len(rids) == 1


def test_small_requests_never_wait_behind_large_ones():
    """With the large lane busy on a stream of large requests, small requests keep flowing
    through the small lanes, and no small lane ever takes a large request."""
    big = [Request(i, 1 << 10, *[a.numpy() for a in graphgen.rmat(10, 16, i)[:2]],
                   arrival=0.0) for i in range(4)]
    small = [Request(100 + i, 200, *[a.numpy() for a in graphgen.erdos_renyi(200, 800, i)[:2]],
                     arrival=1e-4 * i) for i in range(12)]
    ex = FakeExecutor(_lanes(small=2, large=1), polls=6)
    eng = Engine(ex, clock=FakeClock())
    eng.run(big + small, idle_sleep=0)
    assert all(r.total is not None for r in big + small)
    last_small = max(r.done for r in small)
    last_big = max(r.done for r in big)
    assert last_small < last_big  # the small ones are done while large ones still queue
    for lane, rids in ex.launched:
        if not ex.lanes[lane].large:
            assert all(rid >= 100 for rid in rids)


def test_invalid_and_oversized_requests_are_rejected_not_blocking():
    reqs = _requests(6)
    bad = Request(98, 10, np.array([0, 10], np.int32), np.array([1, 2], np.int32), arrival=0.0)
    neg = Request(97, 10, np.array([0, -1], np.int32), np.array([1, 2], np.int32), arrival=0.0)
    big = Request(99, 10**6, np.zeros(10**6, np.int32), np.ones(10**6, np.int32), arrival=0.0)
    assert validate(bad) and validate(neg) and validate(big) is None
    eng = Engine(FakeExecutor(_lanes()), clock=FakeClock())
    st = eng.run([bad, neg, big] + reqs, idle_sleep=0)
    assert st.rejected == 3 and st.completed == 6
    for r in (bad, neg, big):
        assert r.error and r.total is None


def test_device_error_fails_its_batch_only_and_serving_continues():
    reqs = _requests(20)
    reqs[5].fail = True
    ex = FakeExecutor(_lanes(small=1, large=0, graphs=4))
    eng = Engine(ex, clock=FakeClock())
    st = eng.run(reqs, idle_sleep=0)
    bad_batch = next(rids for _, rids in ex.launched if 5 in rids)
    assert st.failed == len(bad_batch) and st.completed == 20 - len(bad_batch)
    for r in reqs:
        if r.rid in bad_batch:
            assert r.error and r.total is None
        else:
            assert r.error is None and r.total is not None
    assert not eng.inflight


def test_fifo_within_a_queue_and_capacity_one_request():
    reqs = _requests(12)
    ex = FakeExecutor(_lanes(small=1, large=0, small_pairs=900), polls=2)
    eng = Engine(ex, clock=FakeClock())
    eng.run(reqs, idle_sleep=0)
    order = [rid for _, rids in ex.launched for rid in rids]
    assert order == sorted(order)
    assert all(len(rids) == 1 for _, rids in ex.launched)


def test_summary_percentiles():
    reqs = _requests(30)
    eng = Engine(FakeExecutor(_lanes()), clock=FakeClock())
    st = eng.run(reqs, idle_sleep=0)
    s = st.summary()
    assert s["completed"] == 30 and s["p50_ms"] <= s["p99_ms"]
    assert s["graphs_per_s"] > 0


def test_summary_splits_small_and_large_requests():
    """Latencies are also reported per class: requests the small lanes take and the large
    ones (admitted to the large lanes' queue)."""
    reqs = _requests(40, large_every=9)
    eng = Engine(FakeExecutor(_lanes()), clock=FakeClock())
    st = eng.run(reqs, idle_sleep=0)
    s = st.summary()
    n_large = sum(r.large for r in reqs)
    assert n_large == sum(r.num_pairs > 4000 for r in reqs) > 0
    assert len(st.large_flags) == len(st.latencies) == 40
    assert s["small_p50_ms"] is not None and s["large_p99_ms"] is not None
    lat = np.array(st.latencies) * 1e3
    big = np.array(st.large_flags)
    assert s["large_p99_ms"] == pytest.approx(np.percentile(lat[big], 99))
    assert s["small_p50_ms"] == pytest.approx(np.percentile(lat[~big], 50))


def test_device_busy_fraction_merges_overlapping_batches():
    from paper_1909_02127_amd.serve import Stats
    st = Stats()
    st.first_arrival, st.last_done = 0.0, 10.0
    st.intervals = [(1.0, 3.0), (2.0, 4.0), (6.0, 7.0), (6.5, 6.8)]
    assert st.summary()["device_busy_frac"] == pytest.approx(0.4)
    reqs = _requests(30)
    eng = Engine(FakeExecutor(_lanes()), clock=FakeClock())
    s = eng.run(reqs, idle_sleep=0).summary()
    assert 0.0 < s["device_busy_frac"] <= 1.0
