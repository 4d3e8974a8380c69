"""Continuous-batching serving loop for triangle-count requests.

A request is one undirected graph (raw int32 pairs with local ids, in host
memory) that asks for its exact total and per-vertex counts.  The engine

  * admits waiting requests in arrival order while their estimated HBM
    footprint fits the budget (a request larger than the whole budget is
    rejected);
  * packs the requests admitted since the last launch into one batch (the
    disjoint union of their graphs) and launches it on a free stream: upload,
    tc_build_csr, tc_orient, tc_count_batched with per-vertex counts, and
    asynchronous copies of the results into pinned host memory, all enqueued
    without host synchronisation, so batches on different streams overlap on
    the device while new requests keep arriving;
  * gives requests above `large_pairs` a lane of their own (one per batch) so a
    large graph does not hold up the small ones behind it;
  * polls the batches' completion events, hands each request its counts,
    releases its memory, and records latency = completion - arrival.

The scheduling logic is independent of the device: `Engine` drives an
executor with launch / ready / collect, so it can be exercised with a fake.
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

    @property
    def num_pairs(self) -> int:
        return int(len(self.src))


def footprint_bytes(n: int, num_pairs: int) -> int:
    """Device bytes a request holds while in flight (its share of a batch): the
    pairs (8 B each), the build keys (2 x 16 B per pair), the symmetric and
    oriented CSR (12 B per pair, 16 B per vertex for int64 offsets), the orientation's
    per-tile state (under 1 B per pair), per-vertex counts and scratch (about 24 B per
    vertex)."""
    return 8 * num_pairs + 32 * num_pairs + 12 * num_pairs + num_pairs + 16 * (n + 1) + 24 * n \
        + 1024


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    completed: int = 0
    rejected: int = 0
    batches: int = 0
    max_in_use: int = 0
    max_inflight_batches: int = 0
    first_arrival: float | None = None
    last_done: float | None = None

    def summary(self, warmup: int = 0) -> dict:
        lat = np.array(self.latencies[warmup:], dtype=np.float64) * 1e3
        span = (self.last_done or 0.0) - (self.first_arrival or 0.0)
        return {
            "completed": self.completed,
            "rejected": self.rejected,
            "batches": self.batches,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            "graphs_per_s": self.completed / span if span > 0 else None,
            "max_in_use_bytes": self.max_in_use,
            "max_inflight_batches": self.max_inflight_batches,
        }


class Engine:
    def __init__(self, executor, *, budget_bytes: int, max_inflight: int = 3,
                 max_batch: int = 1024, large_pairs: int = 8_000_000, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.large_pairs = large_pairs
        self.clock = clock
        self.waiting: collections.deque[Request] = collections.deque()
        self.admitted_small: list[Request] = []
        self.admitted_large: collections.deque[Request] = collections.deque()
        self.inflight: list[tuple[object, list[Request], int, bool]] = []
        self.in_use = 0
        self.stats = Stats()
        self.finished: list[Request] = []

    # -- admission ------------------------------------------------------------------
    def submit(self, req: Request) -> None:
        if self.stats.first_arrival is None or req.arrival < self.stats.first_arrival:
            self.stats.first_arrival = req.arrival
        if footprint_bytes(req.n, req.num_pairs) > self.budget:
            req.error = "request footprint exceeds the device budget"
            req.done = self.clock()
            self.stats.rejected += 1
            self.finished.append(req)
            return
        self.waiting.append(req)

    def _admit(self) -> None:
        while self.waiting:
            req = self.waiting[0]
            need = footprint_bytes(req.n, req.num_pairs)
            if self.in_use + need > self.budget:
                break  # FIFO: later requests wait behind it (no starvation of large ones)
            self.waiting.popleft()
            self.in_use += need
            self.stats.max_in_use = max(self.stats.max_in_use, self.in_use)
            req.admitted = self.clock()
            if req.num_pairs >= self.large_pairs:
                self.admitted_large.append(req)
            else:
                self.admitted_small.append(req)

    # -- launching and completion ---------------------------------------------------------
    def _lanes_busy(self, large: bool) -> int:
        return sum(1 for _, _, _, lg in self.inflight if lg == large)

    def _launch(self) -> None:
        # one lane for large requests, the rest for packed batches of small ones
        if self.admitted_large and self._lanes_busy(True) == 0:
            req = self.admitted_large.popleft()
            self._start([req], True)
        small_lanes = max(1, self.max_inflight - 1)
        while self.admitted_small and self._lanes_busy(False) < small_lanes:
            batch = self.admitted_small[: self.max_batch]
            self.admitted_small = self.admitted_small[self.max_batch:]
            self._start(batch, False)

    def _start(self, reqs: list[Request], large: bool) -> None:
        handle = self.ex.launch(reqs)
        mem = sum(footprint_bytes(r.n, r.num_pairs) for r in reqs)
        self.inflight.append((handle, reqs, mem, large))
        self.stats.batches += 1
        self.stats.max_inflight_batches = max(self.stats.max_inflight_batches, len(self.inflight))

    def _poll(self) -> None:
        still = []
        for handle, reqs, mem, large in self.inflight:
            if not self.ex.ready(handle):
                still.append((handle, reqs, mem, large))
                continue
            totals, per_vertex = self.ex.collect(handle)
            now = self.clock()
            for r, t, pv in zip(reqs, totals, per_vertex):
                r.total, r.per_vertex, r.done = t, pv, now
                self.stats.latencies.append(now - r.arrival)
                self.stats.completed += 1
                self.finished.append(r)
            self.stats.last_done = now
            self.in_use -= mem
        self.inflight = still

    def step(self) -> bool:
        """One engine iteration; returns True while work is queued or in flight."""
        self._poll()
        self._admit()
        self._launch()
        return bool(self.waiting or self.admitted_small or self.admitted_large or self.inflight)

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


class DeviceExecutor:
    """Runs a batch of requests on the GPU through the C ABI, on its own stream."""

    def __init__(self, device="cuda", *, tune=None):
        import torch

        from . import _lib
        self.torch = torch
        self.lib = _lib
        self.device = torch.device(device)
        self.tune = tune
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(4)]
        self.busy = [False] * 4

    def _stream(self):
        for i, b in enumerate(self.busy):
            if not b:
                self.busy[i] = True
                return i
        raise RuntimeError("no free stream")

    def launch(self, reqs: list[Request]):
        torch, L = self.torch, self.lib
        si = self._stream()
        stream = self.streams[si]
        ns = [r.n for r in reqs]
        off = np.zeros(len(reqs) + 1, dtype=np.int64)
        off[1:] = np.cumsum(ns)
        pairs = np.zeros(len(reqs) + 1, dtype=np.int64)
        pairs[1:] = np.cumsum([r.num_pairs for r in reqs])
        n, p, G = int(off[-1]), int(pairs[-1]), len(reqs)
        dev = self.device
        with torch.cuda.stream(stream):
            src = torch.empty(max(p, 1), dtype=torch.int32, device=dev)
            dst = torch.empty(max(p, 1), dtype=torch.int32, device=dev)
            for r, a in zip(reqs, pairs[:-1]):
                k = r.num_pairs
                if k:
                    src[a: a + k].copy_(_pinned(torch, r.src), non_blocking=True)
                    dst[a: a + k].copy_(_pinned(torch, r.dst), non_blocking=True)
            if G > 1 and p:
                shift = torch.repeat_interleave(
                    torch.as_tensor(off[:-1], device=dev),
                    torch.as_tensor(pairs[1:] - pairs[:-1], device=dev))
                src[:p] += shift.to(torch.int32)
                dst[:p] += shift.to(torch.int32)
            vtx_off = torch.as_tensor(off, device=dev)
            row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
            col = torch.empty(max(2 * p, 1), dtype=torch.int32, device=dev)
            nnz = torch.empty(1, dtype=torch.int64, device=dev)
            ws_b = torch.empty(max(L.tc_build_csr_workspace(n, p, 8), 1), dtype=torch.uint8,
                               device=dev)
            L.tc_build_csr(n, src[:p], dst[:p], row_ptr, col, nnz, ws_b, stream=stream)
            dag_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
            dag_col = torch.empty(max(p, 1), dtype=torch.int32, device=dev)
            m = torch.empty(1, dtype=torch.int64, device=dev)
            ws_o = torch.empty(max(L.tc_orient_workspace(n, dag_col.numel()), 1), dtype=torch.uint8,
                               device=dev)
            L.tc_orient(n, row_ptr, col, L.TC_ORDER_DEGREE, dag_ptr, dag_col, m, ws_o,
                        stream=stream)
            totals = torch.empty(max(G, 1), dtype=torch.int64, device=dev)
            pv = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
            ws_c = torch.empty(max(L.tc_count_batched_workspace(n), 1), dtype=torch.uint8,
                               device=dev)
            L.tc_count_batched(n, dag_ptr, dag_col, vtx_off, totals[:G], ws_c,
                               per_vertex=pv[:n], tune=self.tune, stream=stream)
            h_totals = torch.empty(max(G, 1), dtype=torch.int64, pin_memory=True)
            h_pv = torch.empty(max(n, 1), dtype=torch.int64, pin_memory=True)
            h_err = torch.empty(2, dtype=torch.int64, pin_memory=True)
            h_totals.copy_(totals, non_blocking=True)
            h_pv.copy_(pv, non_blocking=True)
            h_err[0:1].copy_(nnz, non_blocking=True)
            h_err[1:2].copy_(m, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        # device buffers stay referenced by the handle until collect()
        keep = (src, dst, vtx_off, row_ptr, col, nnz, ws_b, dag_ptr, dag_col, m, ws_o, totals,
                pv, ws_c)
        return {"ev": ev, "si": si, "G": G, "off": off, "h": (h_totals, h_pv, h_err), "keep": keep}

    def ready(self, handle) -> bool:
        return handle["ev"].query()

    def collect(self, handle):
        h_totals, h_pv, h_err = handle["h"]
        self.busy[handle["si"]] = False
        handle["keep"] = None
        if int(h_err[0]) < 0:
            raise self.lib.TcError(-int(h_err[0]), "reported by tc_build_csr on the device")
        if int(h_err[1]) < 0:
            raise self.lib.TcError(-int(h_err[1]), "reported by tc_orient on the device")
        mask = (1 << 64) - 1
        G, off = handle["G"], handle["off"]
        totals = [x & mask for x in h_totals[:G].tolist()]
        pv_all = h_pv.numpy().view(np.uint64)
        per_vertex = [pv_all[off[i]: off[i + 1]].copy() for i in range(G)]
        return totals, per_vertex


def _pinned(torch, a):
    if isinstance(a, torch.Tensor):
        return a
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32))
