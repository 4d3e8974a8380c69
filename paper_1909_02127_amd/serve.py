"""Continuous-batching serving loop for triangle-count requests.

A request is one undirected graph (raw int32 pairs with local ids, in host
memory) that asks for its exact total and per-vertex counts.  The device side is
a fixed pool of *lanes*, allocated once from the HBM budget and kept resident:
each lane owns a HIP stream and every buffer one batch needs in flight (pairs,
symmetric CSR, oriented DAG, the three workspaces, per-graph totals, per-vertex
counts) plus pinned host buffers for the results, sized for the lane's capacity
in pairs, vertices and graphs.  Launching a batch allocates nothing; it reuses
the lane's buffers.  The engine

  * validates each request on submit (ids inside [0, n)) and routes it by size to
    one of two admission queues: requests that fit a small lane, and larger ones
    that only a large lane holds; a request larger than every lane is rejected;
  * whenever a lane is free, packs the head of its queue (FIFO, as many requests
    as fit the lane's capacity) into one batch and launches it on the lane's
    stream: upload, tc_pack_pairs (local ids -> ids of the disjoint union),
    tc_build_csr, tc_orient, tc_count_batched with per-vertex counts and the
    copies of the results into pinned memory, with no host synchronisation, so
    batches on different lanes overlap on the device while new requests arrive.
    Small requests never queue behind large ones: large lanes take the large
    queue first and small lanes never take large requests;
  * polls the lanes' completion events, hands each request its counts (or the
    batch's device-side error), frees the lane and records latency = completion
    - arrival.

The scheduling logic is independent of the device: `Engine` drives an executor
that exposes its lanes and `launch / ready / collect`, so it is tested on the CPU
with a fake.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    n: int
    src: object  # int32 pairs, host memory (numpy array or pinned torch tensor)
    dst: object
    arrival: float = 0.0  # seconds on the engine clock
    admitted: float | None = None
    done: float | None = None
    total: int | None = None
    per_vertex: np.ndarray | None = None
    error: str | None = None
    large: bool = False  # admitted to the large lanes' queue

    @property
    def num_pairs(self) -> int:
        return int(len(self.src))


@dataclass(frozen=True)
class Lane:
    """Capacity of one preallocated device slot (one batch in flight)."""
    index: int
    large: bool
    max_pairs: int
    max_vertices: int
    max_graphs: int
    bytes: int = 0  # device bytes the lane holds

    def fits(self, pairs: int, vertices: int, graphs: int = 1) -> bool:
        return pairs <= self.max_pairs and vertices <= self.max_vertices and \
            graphs <= self.max_graphs


def _host_array(a) -> np.ndarray:
    if isinstance(a, np.ndarray):
        return a
    return a.numpy()  # a (pinned) CPU torch tensor


def validate(req: Request) -> str | None:
    """Why the request cannot be counted, or None."""
    if req.n < 0:
        return "negative vertex count"
    if len(req.src) != len(req.dst):
        return "src and dst differ in length"
    if req.num_pairs == 0:
        return None
    s, d = _host_array(req.src), _host_array(req.dst)
    lo = min(int(s.min()), int(d.min()))
    hi = max(int(s.max()), int(d.max()))
    if lo < 0 or hi >= req.n:
        return f"vertex id outside [0, {req.n})"
    return None


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    large_flags: list = field(default_factory=list)  # per latency: the request was large
    intervals: list = field(default_factory=list)  # per batch: (launched, seen done) host times
    launch_s: float = 0.0   # host time spent enqueueing batches (copies, kernel launches)
    collect_s: float = 0.0  # host time spent reading batches' results
    completed: int = 0
    rejected: int = 0
    failed: int = 0
    batches: int = 0
    large_batches: int = 0
    max_in_use: int = 0
    max_inflight_batches: int = 0
    first_arrival: float | None = None
    last_done: float | None = None

    def summary(self, warmup: int = 0) -> dict:
        lat = np.array(self.latencies[warmup:], dtype=np.float64) * 1e3
        big = np.array(self.large_flags[warmup:], dtype=bool)
        span = (self.last_done or 0.0) - (self.first_arrival or 0.0)

        def pct(x, q):
            return float(np.percentile(x, q)) if x.size else None

        # the time at least one batch was on the device (launch to its completion being seen)
        busy, end = 0.0, None
        for a, b in sorted(self.intervals):
            if end is None or a > end:
                busy += b - a
                end = b
            elif b > end:
                busy += b - end
                end = b
        return {
            "completed": self.completed,
            "rejected": self.rejected,
            "failed": self.failed,
            "batches": self.batches,
            "large_batches": self.large_batches,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            # the two classes apart: the small lanes' requests and the large ones
            "small_p50_ms": pct(lat[~big], 50) if big.size == lat.size else None,
            "small_p99_ms": pct(lat[~big], 99) if big.size == lat.size else None,
            "large_p50_ms": pct(lat[big], 50) if big.size == lat.size else None,
            "large_p99_ms": pct(lat[big], 99) if big.size == lat.size else None,
            "graphs_per_s": self.completed / span if span > 0 else None,
            "max_in_use_bytes": self.max_in_use,
            "max_inflight_batches": self.max_inflight_batches,
            "device_busy_frac": busy / span if span > 0 else None,
            "host_launch_frac": self.launch_s / span if span > 0 else None,
            "host_collect_frac": self.collect_s / span if span > 0 else None,
        }


class Engine:
    """Admission, batching and completion over an executor's lanes."""

    def __init__(self, executor, *, clock=time.perf_counter):
        self.ex = executor
        self.lanes: list[Lane] = list(executor.lanes)
        if not self.lanes:
            raise ValueError("the executor has no lanes")
        self.clock = clock
        self.small_q: collections.deque[Request] = collections.deque()
        self.large_q: collections.deque[Request] = collections.deque()
        self.inflight: dict[int, tuple[object, list[Request], float]] = {}  # lane -> (handle, reqs, launched)
        self.stats = Stats()
        self.finished: list[Request] = []
        small = [ln for ln in self.lanes if not ln.large]
        large = [ln for ln in self.lanes if ln.large]
        self._small_cap = small[0] if small else None
        self._large_caps = large

    # -- admission ------------------------------------------------------------------
    def _finish_now(self, req: Request, error: str, rejected: bool) -> None:
        req.error = error
        req.done = self.clock()
        if rejected:
            self.stats.rejected += 1
        else:
            self.stats.failed += 1
        self.finished.append(req)

    def submit(self, req: Request) -> None:
        if self.stats.first_arrival is None or req.arrival < self.stats.first_arrival:
            self.stats.first_arrival = req.arrival
        why = validate(req)
        if why is not None:
            self._finish_now(req, why, True)
            return
        if self._small_cap is not None and self._small_cap.fits(req.num_pairs, req.n):
            self.small_q.append(req)
        elif any(ln.fits(req.num_pairs, req.n) for ln in self._large_caps):
            req.large = True
            self.large_q.append(req)
        else:
            self._finish_now(req, "request is larger than every lane of the device pool", True)

    # -- launching and completion ---------------------------------------------------------
    def _take(self, q: collections.deque, lane: Lane) -> list[Request]:
        batch, pairs, verts = [], 0, 0
        while q and len(batch) < lane.max_graphs:
            r = q[0]
            if not lane.fits(pairs + r.num_pairs, verts + r.n, len(batch) + 1):
                break
            q.popleft()
            batch.append(r)
            pairs += r.num_pairs
            verts += r.n
        return batch

    def _launch(self) -> None:
        for lane in self.lanes:
            if lane.index in self.inflight:
                continue
            batch = []
            if lane.large and self.large_q:
                batch = self._take(self.large_q, lane)
            if not batch and self.small_q:
                batch = self._take(self.small_q, lane)
            if not batch:
                continue
            now = self.clock()
            for r in batch:
                r.admitted = now
            handle = self.ex.launch(lane.index, batch)
            self.stats.launch_s += self.clock() - now
            self.inflight[lane.index] = (handle, batch, now)
            self.stats.batches += 1
            self.stats.large_batches += int(lane.large)
            self.stats.max_inflight_batches = max(self.stats.max_inflight_batches,
                                                  len(self.inflight))
            in_use = sum(self.lanes[i].bytes for i in self.inflight)
            self.stats.max_in_use = max(self.stats.max_in_use, in_use)

    def _poll(self) -> None:
        for li in list(self.inflight):
            handle, reqs, launched = self.inflight[li]
            if not self.ex.ready(handle):
                continue
            t0 = self.clock()
            totals, per_vertex, error = self.ex.collect(handle)
            del self.inflight[li]
            now = self.clock()
            self.stats.collect_s += now - t0
            self.stats.intervals.append((launched, now))
            for k, r in enumerate(reqs):
                r.done = now
                if error is not None:
                    r.error = error
                    self.stats.failed += 1
                else:
                    r.total, r.per_vertex = totals[k], per_vertex[k]
                    self.stats.latencies.append(now - r.arrival)
                    self.stats.large_flags.append(r.large)
                    self.stats.completed += 1
                self.finished.append(r)
            self.stats.last_done = now

    def busy(self) -> bool:
        return bool(self.small_q or self.large_q or self.inflight)

    def step(self) -> bool:
        """One engine iteration; returns True while work is queued or in flight."""
        self._poll()
        self._launch()
        return self.busy()

    def run(self, requests: list[Request], *, idle_sleep: float = 50e-6) -> Stats:
        """Open-loop run: each request is submitted once the clock passes its arrival
        time (given relative to the start of the run; stored back as absolute)."""
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = self.clock()
        for r in order:
            r.arrival += t0
        i = 0
        while True:
            now = self.clock()
            while i < len(order) and order[i].arrival <= now:
                self.submit(order[i])
                i += 1
            busy = self.step()
            if not busy and i >= len(order):
                break
            if not busy:
                wait = order[i].arrival - self.clock()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            elif idle_sleep:
                time.sleep(idle_sleep)
        return self.stats


def lane_bytes(lib, max_pairs: int, max_vertices: int, max_graphs: int) -> int:
    """Device bytes of one lane: pairs, symmetric CSR and DAG with int64 offsets, the
    three workspaces at capacity, graph offsets, totals and per-vertex counts."""
    n, p, g = max_vertices, max_pairs, max_graphs
    b = 8 * p                                    # src, dst
    b += 8 * (n + 1) + 4 * 2 * p                 # row_ptr, col
    b += 8 * (n + 1) + 4 * p                     # dag_ptr, dag_col
    b += 16 * (g + 1) + 8 * g + 8 * n + 64       # pair/vtx offsets, totals, per-vertex, sizes
    b += lib.tc_build_csr_workspace(n, p, 8)
    b += lib.tc_orient_workspace(n, p)
    b += lib.tc_count_batched_workspace(n)
    return int(b)


def plan_lanes(lib, budget_bytes: int, *, small_lanes: int = 3, small_pairs: int = 32_000_000,
               small_vertices: int = 8_000_000, small_graphs: int = 512, large_lanes: int = 1,
               large_pairs: int = 70_000_000, large_vertices: int = 1 << 22) -> list[Lane]:
    """The lane pool: large lanes (index 0 ...) holding graphs of up to large_pairs pairs
    on large_vertices vertices together, then small lanes holding up to small_graphs graphs
    with small_pairs pairs on small_vertices vertices together.  A large lane takes large
    requests first and, when none is queued, a batch of small ones (up to small_graphs).
    Raises ValueError when the pool does not fit `budget_bytes` of device memory."""
    lanes = []
    for _ in range(large_lanes):
        lanes.append(Lane(len(lanes), True, large_pairs, large_vertices, small_graphs,
                          lane_bytes(lib, large_pairs, large_vertices, small_graphs)))
    for _ in range(small_lanes):
        lanes.append(Lane(len(lanes), False, small_pairs, small_vertices, small_graphs,
                          lane_bytes(lib, small_pairs, small_vertices, small_graphs)))
    total = sum(ln.bytes for ln in lanes)
    if total > budget_bytes:
        raise ValueError(f"the lane pool needs {total} bytes, above the budget of {budget_bytes}")
    return lanes


class DeviceExecutor:
    """Runs batches on the GPU through the C ABI, one resident lane per batch in flight."""

    def __init__(self, lanes: list[Lane], device="cuda", *, tune=None, large_tune=None):
        """tune: tc_tune of the small lanes' counts; large_tune: of the large lanes' (None:
        tune).  A large lane's count is one persistent launch over every CU; a smaller grid
        (blocks_per_cu) leaves workgroup slots to the small lanes' batches meanwhile."""
        import torch

        from . import _lib
        self.torch = torch
        self.lib = _lib
        self.device = torch.device(device)
        self.tune = tune
        self.large_tune = tune if large_tune is None else large_tune
        self.lanes = list(lanes)
        self.slots = [self._alloc(ln) for ln in self.lanes]

    def _alloc(self, ln: Lane) -> dict:
        torch, L, dev = self.torch, self.lib, self.device
        p, n, g = max(ln.max_pairs, 1), max(ln.max_vertices, 1), max(ln.max_graphs, 1)

        def dbuf(k, dt):
            return torch.empty(k, dtype=dt, device=dev)

        def hbuf(k, dt):
            return torch.empty(k, dtype=dt, pin_memory=True)

        return {
            "stream": torch.cuda.Stream(device=dev),
            "event": torch.cuda.Event(),
            "src": dbuf(p, torch.int32), "dst": dbuf(p, torch.int32),
            "row_ptr": dbuf(n + 1, torch.int64), "col": dbuf(2 * p, torch.int32),
            "dag_ptr": dbuf(n + 1, torch.int64), "dag_col": dbuf(p, torch.int32),
            "offs": dbuf(2 * (g + 1), torch.int64),  # pair offsets, then vertex offsets
            "totals": dbuf(g, torch.int64), "pv": dbuf(n, torch.int64),
            "sizes": dbuf(2, torch.int64),  # nnz, m
            "ws_build": dbuf(L.tc_build_csr_workspace(n, p, 8), torch.uint8),
            "ws_orient": dbuf(L.tc_orient_workspace(n, p), torch.uint8),
            "ws_count": dbuf(L.tc_count_batched_workspace(n), torch.uint8),
            "h_src": hbuf(p, torch.int32), "h_dst": hbuf(p, torch.int32),
            "h_offs": hbuf(2 * (g + 1), torch.int64),
            "h_totals": hbuf(g, torch.int64), "h_pv": hbuf(n, torch.int64),
            "h_sizes": hbuf(2, torch.int64),
        }

    def launch(self, lane_index: int, reqs: list[Request]):
        torch, L = self.torch, self.lib
        b = self.slots[lane_index]
        G = len(reqs)
        poff = np.zeros(G + 1, dtype=np.int64)
        poff[1:] = np.cumsum([r.num_pairs for r in reqs])
        voff = np.zeros(G + 1, dtype=np.int64)
        voff[1:] = np.cumsum([r.n for r in reqs])
        p, n = int(poff[-1]), int(voff[-1])
        h_offs = b["h_offs"].numpy()
        h_offs[: G + 1] = poff
        h_offs[G + 1: 2 * G + 2] = voff
        stream = b["stream"]
        with torch.cuda.stream(stream):
            for r, a in zip(reqs, poff[:-1]):
                k = r.num_pairs
                if not k:
                    continue
                for key, arr in (("src", r.src), ("dst", r.dst)):
                    if isinstance(arr, torch.Tensor) and arr.is_pinned():
                        b[key][a: a + k].copy_(arr, non_blocking=True)
                    else:  # stage through the lane's pinned buffer
                        h = b["h_" + key]
                        h.numpy()[a: a + k] = _host_array(arr)
                        b[key][a: a + k].copy_(h[a: a + k], non_blocking=True)
            offs = b["offs"]
            offs[: 2 * G + 2].copy_(b["h_offs"][: 2 * G + 2], non_blocking=True)
            pair_off, vtx_off = offs[: G + 1], offs[G + 1: 2 * G + 2]
            if G > 1:
                L.tc_pack_pairs(pair_off, vtx_off, b["src"][:p], b["dst"][:p], stream=stream)
            sizes = b["sizes"]
            # output capacities of this batch (not of the lane): the orientation's tiles and
            # scan are sized by them
            q = max(p, 1)
            L.tc_build_csr(n, b["src"][:p], b["dst"][:p], b["row_ptr"][: n + 1],
                           b["col"][: 2 * q], sizes[0:1], b["ws_build"], stream=stream)
            L.tc_orient(n, b["row_ptr"][: n + 1], b["col"][: 2 * q], L.TC_ORDER_DEGREE,
                        b["dag_ptr"][: n + 1], b["dag_col"][:q], sizes[1:2], b["ws_orient"],
                        stream=stream)
            L.tc_count_batched(n, b["dag_ptr"][: n + 1], b["dag_col"], vtx_off, b["totals"][:G],
                               b["ws_count"], per_vertex=b["pv"][:n],
                               tune=self.large_tune if self.lanes[lane_index].large else self.tune,
                               stream=stream)
            b["h_totals"][:G].copy_(b["totals"][:G], non_blocking=True)
            b["h_pv"][:n].copy_(b["pv"][:n], non_blocking=True)
            b["h_sizes"].copy_(sizes, non_blocking=True)
            b["event"].record(stream)
        return {"lane": lane_index, "G": G, "voff": voff}

    def ready(self, handle) -> bool:
        return self.slots[handle["lane"]]["event"].query()

    def collect(self, handle):
        """(totals, per-vertex arrays, error): a device-side error fails the whole batch."""
        b = self.slots[handle["lane"]]
        G, voff = handle["G"], handle["voff"]
        nnz, m = (int(x) for x in b["h_sizes"].tolist())
        if nnz < 0:
            return None, None, f"tc_build_csr: {self.lib.status_string(-nnz)}"
        if m < 0:
            return None, None, f"tc_orient: {self.lib.status_string(-m)}"
        mask = (1 << 64) - 1
        totals = [x & mask for x in b["h_totals"][:G].tolist()]
        pv_all = b["h_pv"].numpy().view(np.uint64)
        per_vertex = [pv_all[voff[i]: voff[i + 1]].copy() for i in range(G)]
        return totals, per_vertex, None
