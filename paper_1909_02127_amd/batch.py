"""Batched counting of many independent graphs on one GPU.

A batch is the disjoint union of its graphs with global vertex ids: graph g owns
ids [vtx_off[g], vtx_off[g+1]).  It is built once with tc_build_csr from the
concatenated, id-shifted pairs, and counted with tc_orient + tc_count_batched:
a fixed sequence of about fifteen kernel launches for the whole batch, which
`BatchRunner.capture()` records into a HIP graph for replay.

For comparison, `PlainRunner` runs the one-graph-per-launch path: tc_orient +
tc_count on each graph's own CSR, all on one stream without host synchronisation.
"""
from __future__ import annotations

import torch

from . import _lib
from .pipeline import _bytes


class PackedBatch:
    """Union CSR of G graphs given as lists of per-graph (src, dst, n) with local ids."""

    def __init__(self, graphs, *, device="cuda", offset_bytes: int | None = None):
        """offset_bytes: width of the union's row offsets; None picks 4 when the symmetric
        union fits int32 offsets (2 * pairs < 2^31), else 8."""
        dev = torch.device(device)
        self.device = dev
        ns = [int(n) for _, _, n in graphs]
        self.G = len(graphs)
        off = [0]
        for n in ns:
            off.append(off[-1] + n)
        self.n = off[-1]
        self.vtx_off = torch.tensor(off, dtype=torch.int64, device=dev)
        src = torch.cat([s.to(dev, torch.int64) + o for (s, _, _), o in zip(graphs, off)]) \
            if graphs else torch.zeros(0, dtype=torch.int64, device=dev)
        dst = torch.cat([d.to(dev, torch.int64) + o for (_, d, _), o in zip(graphs, off)]) \
            if graphs else torch.zeros(0, dtype=torch.int64, device=dev)
        self.num_pairs = src.numel()
        if offset_bytes is None:
            offset_bytes = 4 if 2 * self.num_pairs < 2**31 else 8
        self.offset_bytes = offset_bytes
        src, dst = src.to(torch.int32), dst.to(torch.int32)
        odt = torch.int32 if offset_bytes == 4 else torch.int64
        self.offset_dtype = odt
        self.row_ptr = torch.empty(self.n + 1, dtype=odt, device=dev)
        self.col = torch.empty(max(2 * self.num_pairs, 1), dtype=torch.int32, device=dev)
        nnz = torch.zeros(1, dtype=torch.int64, device=dev)
        ws = _bytes(_lib.tc_build_csr_workspace(self.n, self.num_pairs, offset_bytes), dev)
        _lib.tc_build_csr(self.n, src, dst, self.row_ptr, self.col, nnz, ws)
        torch.cuda.synchronize(dev)
        self.nnz = int(nnz.item())
        if self.nnz < 0:
            raise _lib.TcError(-self.nnz, "reported by tc_build_csr on the device")
        del ws, src, dst
        self.col = self.col[: max(self.nnz, 1)].clone()
        self.m = self.nnz // 2
        self.graph_m = None

    def graph_edges(self) -> list[int]:
        """Undirected edges of every graph (one host read)."""
        if self.graph_m is None:
            starts = self.row_ptr[self.vtx_off].to(torch.int64)
            self.graph_m = ((starts[1:] - starts[:-1]) // 2).cpu().tolist()
        return self.graph_m

    def local_csr(self):
        """Each graph as its own CSR with local ids, packed back to back: returns
        (row_ptr_local int64[sum(n_g + 1)], col_local int32[nnz], views) where views[g]
        = (n_g, row slice, col slice)."""
        rp = self.row_ptr.to(torch.int64)
        col = self.col[: self.nnz].to(torch.int64)
        off = self.vtx_off.cpu().tolist()
        ebeg = rp[self.vtx_off].cpu().tolist()
        rp_local = torch.empty(self.n + self.G, dtype=torch.int64, device=self.device)
        col_local = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        views = []
        for g in range(self.G):
            a, b = off[g], off[g + 1]
            r = rp_local[a + g: b + g + 1]
            r.copy_(rp[a: b + 1] - ebeg[g])
            c = col_local[ebeg[g]: ebeg[g + 1]]
            c.copy_((col[ebeg[g]: ebeg[g + 1]] - a).to(torch.int32))
            views.append((b - a, r, c))
        return rp_local, col_local, views


class BatchRunner:
    """tc_orient + tc_count_batched over a PackedBatch; optionally captured in a HIP graph."""

    def __init__(self, batch: PackedBatch, *, per_vertex: bool = False, tune=None,
                 order: int = _lib.TC_ORDER_DEGREE):
        self.b = batch
        dev = batch.device
        self.per_vertex = per_vertex
        self.tune = tune
        self.order = order
        self.dag_ptr = torch.empty(batch.n + 1, dtype=batch.offset_dtype, device=dev)
        self.dag_col = torch.empty(max(batch.m, 1), dtype=torch.int32, device=dev)
        self.m_out = torch.zeros(1, dtype=torch.int64, device=dev)
        self.totals = torch.zeros(max(batch.G, 1), dtype=torch.int64, device=dev)
        self.total = torch.zeros(1, dtype=torch.int64, device=dev)
        self.pv = torch.zeros(max(batch.n, 1), dtype=torch.int64, device=dev) if per_vertex else None
        self.ws_orient = _bytes(_lib.tc_orient_workspace(batch.n, self.dag_col.numel()), dev)
        self.ws_count = _bytes(_lib.tc_count_batched_workspace(batch.n), dev)
        self.graph = None

    def enqueue(self) -> None:
        b = self.b
        _lib.tc_orient(b.n, b.row_ptr, b.col, self.order, self.dag_ptr, self.dag_col, self.m_out,
                       self.ws_orient)
        self.count_only()

    def count_only(self) -> None:
        b = self.b
        _lib.tc_count_batched(b.n, self.dag_ptr, self.dag_col, b.vtx_off, self.totals[: b.G],
                              self.ws_count, per_vertex=None if self.pv is None else self.pv[: b.n],
                              total=self.total, tune=self.tune)

    def capture(self) -> None:
        """Record enqueue() into a HIP graph (warm-up run first, outside the capture)."""
        self.enqueue()
        torch.cuda.synchronize(self.b.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.enqueue()
        self.graph = g

    def replay(self) -> None:
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def results(self):
        torch.cuda.synchronize(self.b.device)
        if int(self.m_out.item()) < 0:
            raise _lib.TcError(-int(self.m_out.item()), "reported by tc_orient on the device")
        mask = (1 << 64) - 1
        totals = [x & mask for x in self.totals[: self.b.G].cpu().tolist()]
        return totals, int(self.total.item()) & mask


class PlainRunner:
    """The one-graph-per-launch path: tc_orient + tc_count per graph, one stream, no syncs."""

    def __init__(self, batch: PackedBatch, *, order: int = _lib.TC_ORDER_DEGREE):
        self.b = batch
        dev = batch.device
        self.order = order
        self.rp_local, self.col_local, self.views = batch.local_csr()
        nmax = max([v[0] for v in self.views], default=0)
        self.dag_ptr = torch.empty(batch.n + batch.G, dtype=torch.int64, device=dev)
        self.dag_col = torch.empty(max(batch.m, 1), dtype=torch.int32, device=dev)
        self.m_out = torch.zeros(max(batch.G, 1), dtype=torch.int64, device=dev)
        self.totals = torch.zeros(max(batch.G, 1), dtype=torch.int64, device=dev)
        mmax = max([v[2].numel() // 2 for v in self.views], default=0)
        self.ws_orient = _bytes(_lib.tc_orient_workspace(nmax, mmax), dev)
        self.ws_count = _bytes(_lib.tc_count_workspace(nmax), dev)
        # per-graph DAG slices: rows at the same place as the local CSR, edges packed
        off = batch.vtx_off.cpu().tolist()
        ebeg = [0]
        for g in range(batch.G):
            ebeg.append(ebeg[-1] + self.views[g][2].numel() // 2)
        self.dag_views = []
        for g in range(batch.G):
            n = self.views[g][0]
            self.dag_views.append((self.dag_ptr[off[g] + g: off[g + 1] + g + 1],
                                   self.dag_col[ebeg[g]: ebeg[g + 1]] if ebeg[g + 1] > ebeg[g]
                                   else self.dag_col[:0]))

    def enqueue(self) -> None:
        for g, (n, rp, col) in enumerate(self.views):
            dp, dc = self.dag_views[g]
            _lib.tc_orient(n, rp, col, self.order, dp, dc, self.m_out[g: g + 1], self.ws_orient)
            _lib.tc_count(n, dp, dc, self.totals[g: g + 1], self.ws_count)

    def results(self):
        torch.cuda.synchronize(self.b.device)
        if int(self.m_out[: self.b.G].min().item()) < 0:
            raise _lib.TcError(_lib.TC_ERR_CAPACITY, "reported by tc_orient on the device")
        mask = (1 << 64) - 1
        return [x & mask for x in self.totals[: self.b.G].cpu().tolist()]
