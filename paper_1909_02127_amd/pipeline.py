"""Device pipeline over the C ABI: raw pairs -> CSR -> oriented DAG -> counts.

Buffers and workspaces are allocated once with torch (device memory only) and
reused; every step is a libtc call enqueued on the current stream, so a run has
no host synchronisation until results are read.  Device-side errors reported by
the library (an out-of-range id, an output too small) are raised on read.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import _lib
from ._lib import TC_ORDER_DEGREE, TC_ORDER_ID, TcError  # noqa: F401


def _bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


@dataclass
class Result:
    total: int
    per_vertex: torch.Tensor | None
    nnz: int  # stored entries of the symmetric CSR (2m)
    m: int    # undirected edges = DAG edges


class Pipeline:
    """Preallocated buffers for graphs with up to `num_pairs` raw pairs on `n` vertices.
    `tune` (a tc_tune dict or struct) is the default launch configuration of the count
    calls."""

    def __init__(self, n: int, num_pairs: int, *, offset_bytes: int = 4,
                 order: int = TC_ORDER_DEGREE, device="cuda", tune=None):
        self.n, self.num_pairs, self.order = int(n), int(num_pairs), order
        self.tune = tune
        self.device = torch.device(device)
        odt = torch.int32 if offset_bytes == 4 else torch.int64
        dev = self.device
        self.row_ptr = torch.empty(n + 1, dtype=odt, device=dev)
        self.col = torch.empty(max(2 * num_pairs, 1), dtype=torch.int32, device=dev)
        self.dag_ptr = torch.empty(n + 1, dtype=odt, device=dev)
        self.dag_col = torch.empty(max(num_pairs, 1), dtype=torch.int32, device=dev)
        self.nnz = torch.zeros(1, dtype=torch.int64, device=dev)
        self.m = torch.zeros(1, dtype=torch.int64, device=dev)
        self.total = torch.zeros(1, dtype=torch.int64, device=dev)
        self.per_vertex = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
        self.ws_build = _bytes(_lib.tc_build_csr_workspace(n, num_pairs, offset_bytes), dev)
        self.ws_orient = _bytes(_lib.tc_orient_workspace(n, self.dag_col.numel()), dev)
        self.triples = None
        self.ws_list = None
        self.support = None
        self.ws_support = None
        self.support_m = torch.zeros(1, dtype=torch.int64, device=dev)
        self.ws_intersect = None
        self.ws_diamonds = None
        self.diamond_total = torch.zeros(1, dtype=torch.int64, device=dev)
        self.list_count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.ws_labelled = None
        self.direction = None
        self.edge_label = None
        self.edge_label_m = torch.zeros(1, dtype=torch.int64, device=dev)
        self.edge_labelled_total = torch.zeros(1, dtype=torch.int64, device=dev)
        self.edge_labelled_kept = torch.zeros(1, dtype=torch.int64, device=dev)
        self.ws_edge_labelled = None
        self.direction_m = torch.zeros(1, dtype=torch.int64, device=dev)
        self.directed_total = torch.zeros(1, dtype=torch.int64, device=dev)
        self.labelled_total = torch.zeros(1, dtype=torch.int64, device=dev)
        self.labelled_kept = torch.zeros(1, dtype=torch.int64, device=dev)
        self.ws_count = _bytes(max(_lib.tc_count_workspace(n),
                                   _lib.tc_count_per_vertex_workspace(n)), dev)

    # -- the steps, each one C ABI call --------------------------------------------------
    def build(self, src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
        if src.numel() > self.num_pairs:
            raise ValueError("more pairs than the pipeline was sized for")
        _lib.tc_build_csr(self.n, src, dst, self.row_ptr, self.col, self.nnz, self.ws_build,
                          stream=stream)

    def orient(self, stream=None) -> None:
        _lib.tc_orient(self.n, self.row_ptr, self.col, self.order, self.dag_ptr, self.dag_col,
                       self.m, self.ws_orient, stream=stream)

    def count(self, stream=None, tune=None) -> None:
        tune = self.tune if tune is None else tune
        _lib.tc_count(self.n, self.dag_ptr, self.dag_col, self.total, self.ws_count, tune=tune,
                      stream=stream)

    def count_per_vertex(self, stream=None, tune=None) -> None:
        tune = self.tune if tune is None else tune
        pv = self.per_vertex[: self.n]
        _lib.tc_count_per_vertex(self.n, self.dag_ptr, self.dag_col, pv, self.total,
                                 self.ws_count, tune=tune, stream=stream)

    def list_triangles(self, capacity: int, stream=None, tune=None) -> None:
        """Enqueue tc_list_triangles on the current DAG into a (capacity, 3) buffer that is
        kept across calls (grown when a larger capacity is asked for)."""
        capacity = int(capacity)
        tune = self.tune if tune is None else tune
        if self.triples is None or self.triples.shape[0] < capacity:
            self.triples = torch.empty((max(capacity, 1), 3), dtype=torch.int32,
                                       device=self.device)
        if self.ws_list is None:
            self.ws_list = _bytes(_lib.tc_list_triangles_workspace(self.n), self.device)
        _lib.tc_list_triangles(self.n, self.dag_ptr, self.dag_col, self.triples[:capacity],
                               self.list_count, self.ws_list, tune=tune, stream=stream)

    def edge_support(self, stream=None, tune=None) -> None:
        """Enqueue tc_edge_support on the current DAG (one uint32 count per DAG edge)."""
        tune = self.tune if tune is None else tune
        if self.support is None:
            self.support = torch.empty(self.dag_col.numel(), dtype=torch.int32, device=self.device)
        if self.ws_support is None:
            self.ws_support = _bytes(_lib.tc_edge_support_workspace(self.n), self.device)
        _lib.tc_edge_support(self.n, self.dag_ptr, self.dag_col, self.support, self.support_m,
                             self.ws_support, total=self.total, tune=tune, stream=stream)

    def intersect(self, *, support: bool = False, stream=None) -> None:
        """Enqueue tc_segmented_intersect (merge-path N+(u) & N+(v) for every DAG edge) on
        the current DAG: the total into self.total and, with support, every edge's
        triangles into self.support (read with supports())."""
        cap = self.dag_col.numel()
        if self.ws_intersect is None:
            self.ws_intersect = _bytes(_lib.tc_segmented_intersect_workspace(self.n, cap),
                                       self.device)
        if support and self.support is None:
            self.support = torch.empty(cap, dtype=torch.int32, device=self.device)
        _lib.tc_segmented_intersect(self.n, self.dag_ptr, self.dag_col, self.total,
                                    self.support_m, self.ws_intersect,
                                    support=self.support if support else None, stream=stream)

    def diamonds(self, stream=None, tune=None) -> None:
        """Enqueue tc_count_diamonds on the current DAG (result in self.diamond_total)."""
        tune = self.tune if tune is None else tune
        if self.ws_diamonds is None:
            self.ws_diamonds = _bytes(
                _lib.tc_count_diamonds_workspace(self.n, self.dag_col.numel()), self.device)
        _lib.tc_count_diamonds(self.n, self.dag_ptr, self.dag_col, self.diamond_total,
                               self.support_m, self.ws_diamonds, tune=tune, stream=stream)

    def labelled(self, labels: torch.Tensor, query, stream=None, tune=None) -> None:
        """Enqueue tc_count_labelled on the current DAG: the triangles whose vertex labels
        equal `query` (three labels, any order) into self.labelled_total, the DAG edges
        whose labels fit the query into self.labelled_kept (read with labelled_count())."""
        tune = self.tune if tune is None else tune
        if self.ws_labelled is None:
            self.ws_labelled = _bytes(_lib.tc_count_labelled_workspace(
                self.n, self.dag_col.numel(), self.dag_ptr.element_size()), self.device)
        _lib.tc_count_labelled(self.n, self.dag_ptr, self.dag_col, labels, query,
                               self.labelled_total, self.ws_labelled,
                               kept_out=self.labelled_kept, tune=tune, stream=stream)

    def labelled_count(self) -> int:
        """Synchronise and read the result of labelled()."""
        torch.cuda.synchronize(self.device)
        kept = int(self.labelled_kept.item())
        if kept < 0:
            raise TcError(-kept, "reported by tc_count_labelled on the device")
        return int(self.labelled_total.item()) & ((1 << 64) - 1)

    def edge_directions(self, src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
        """Enqueue tc_edge_directions: the arcs src[i] -> dst[i] (the pairs given to build)
        recorded on the current DAG's edges, for directed()."""
        cap = self.dag_col.numel()
        if self.direction is None:
            self.direction = torch.zeros((cap + 3) // 4 * 4, dtype=torch.uint8,
                                         device=self.device)
        _lib.tc_edge_directions(self.n, self.dag_ptr, self.dag_col, src, dst, self.direction,
                                self.direction_m, stream=stream)

    def directed(self, pattern, *, induced: bool = False, stream=None, tune=None) -> None:
        """Enqueue tc_count_directed on the current DAG and the directions recorded by
        edge_directions(): result in self.directed_total (read with directed_count())."""
        tune = self.tune if tune is None else tune
        if self.direction is None:
            raise RuntimeError("edge_directions() must run first")
        _lib.tc_count_directed(self.n, self.dag_ptr, self.dag_col, self.direction, pattern,
                               self.directed_total, self.ws_count, induced=induced, tune=tune,
                               stream=stream)

    def edge_labels(self, src: torch.Tensor, dst: torch.Tensor, labels: torch.Tensor,
                    stream=None) -> None:
        """Enqueue tc_edge_labels: the labels (uint8, 0..3) of the pairs given to build
        recorded on the current DAG's edges, for edge_labelled()."""
        cap = self.dag_col.numel()
        if self.edge_label is None:
            self.edge_label = torch.zeros((cap + 3) // 4 * 4, dtype=torch.uint8,
                                          device=self.device)
        _lib.tc_edge_labels(self.n, self.dag_ptr, self.dag_col, src, dst, labels,
                            self.edge_label, self.edge_label_m, stream=stream)

    def edge_labelled(self, query, *, stream=None, tune=None) -> None:
        """Enqueue tc_count_edge_labelled (edge labels recorded by edge_labels()): result in
        self.edge_labelled_total (read with edge_labelled_count())."""
        tune = self.tune if tune is None else tune
        if self.edge_label is None:
            raise RuntimeError("edge_labels() must run first")
        if self.ws_edge_labelled is None:
            self.ws_edge_labelled = _bytes(_lib.tc_count_edge_labelled_workspace(
                self.n, self.dag_col.numel(), self.dag_ptr.element_size()), self.device)
        _lib.tc_count_edge_labelled(self.n, self.dag_ptr, self.dag_col, self.edge_label, query,
                                    self.edge_labelled_total, self.ws_edge_labelled,
                                    kept_out=self.edge_labelled_kept, tune=tune, stream=stream)

    def edge_labelled_count(self) -> int:
        """Synchronise and read the result of edge_labelled() (raises when the labels
        reported an error)."""
        torch.cuda.synchronize(self.device)
        em = int(self.edge_label_m.item())
        if em < 0:
            raise TcError(-em, "reported by tc_edge_labels on the device")
        kept = int(self.edge_labelled_kept.item())
        if kept < 0:
            raise TcError(-kept, "reported by tc_count_edge_labelled on the device")
        return int(self.edge_labelled_total.item()) & ((1 << 64) - 1)

    def directed_count(self) -> int:
        """Synchronise and read the result of directed() (raises when the directions reported
        an error)."""
        torch.cuda.synchronize(self.device)
        dm = int(self.direction_m.item())
        if dm < 0:
            raise TcError(-dm, "reported by tc_edge_directions on the device")
        return int(self.directed_total.item()) & ((1 << 64) - 1)

    def diamond_count(self) -> int:
        """Synchronise and read the result of diamonds()."""
        torch.cuda.synchronize(self.device)
        m = int(self.support_m.item())
        if m < 0:
            raise TcError(-m, "reported by tc_count_diamonds on the device")
        return int(self.diamond_total.item()) & ((1 << 64) - 1)

    def intersect_total(self) -> int:
        """Synchronise and read the total written by intersect(); raises TcError when the
        DAG had more edges than the column capacity."""
        torch.cuda.synchronize(self.device)
        m = int(self.support_m.item())
        if m < 0:
            raise TcError(-m, "reported by tc_segmented_intersect on the device")
        return int(self.total.item()) & ((1 << 64) - 1)

    def supports(self) -> torch.Tensor:
        """Synchronise and return the per-edge supports written by edge_support (int32 view
        of the uint32 counts, aligned with dag_col)."""
        torch.cuda.synchronize(self.device)
        m = int(self.support_m.item())
        if m < 0:
            raise TcError(-m, "reported by tc_edge_support on the device")
        return self.support[:m]

    def listing(self) -> torch.Tensor:
        """Synchronise and return the rows written by list_triangles (a view)."""
        torch.cuda.synchronize(self.device)
        c = int(self.list_count.item())
        if c < 0:
            raise TcError(-c, "reported by tc_list_triangles on the device")
        return self.triples[:c]

    def enqueue(self, src, dst, *, per_vertex: bool = False, stream=None) -> None:
        self.build(src, dst, stream)
        self.orient(stream)
        if per_vertex:
            self.count_per_vertex(stream)
        else:
            self.count(stream)

    def result(self, *, per_vertex: bool = False) -> Result:
        """Synchronise and read the counts; raises TcError on a device-side error."""
        torch.cuda.synchronize(self.device)
        nnz, m = int(self.nnz.item()), int(self.m.item())
        if nnz < 0:
            raise TcError(-nnz, "reported by tc_build_csr on the device")
        if m < 0:
            raise TcError(-m, "reported by tc_orient on the device")
        total = int(self.total.item()) & ((1 << 64) - 1)  # the library writes a uint64
        pv = self.per_vertex[: self.n].clone() if per_vertex else None
        return Result(total, pv, nnz, m)


def triangle_count(src: torch.Tensor, dst: torch.Tensor, n: int, *, per_vertex: bool = False,
                   order: int = TC_ORDER_DEGREE, offset_bytes: int = 4, tune=None) -> Result:
    """One-shot count of a raw pair list already in device memory."""
    p = Pipeline(n, src.numel(), offset_bytes=offset_bytes, order=order, device=src.device,
                 tune=tune)
    p.enqueue(src, dst, per_vertex=per_vertex)
    return p.result(per_vertex=per_vertex)
