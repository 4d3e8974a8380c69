"""ctypes binding of libtc.so: the C ABI entry points under their own names.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Torch tensors supply device memory and torch's current stream supplies
the HIP stream.  There is no fallback: if libtc.so is missing, importing this
module raises.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import torch

_LIB_PATH = Path(__file__).resolve().parent / "libtc.so"

TC_OK = 0
TC_ERR_INVALID_ARG = 1
TC_ERR_ID_OUT_OF_RANGE = 2
TC_ERR_CAPACITY = 3
TC_ERR_WORKSPACE = 4
TC_ERR_HIP = 5
TC_ERR_UNSUPPORTED = 6

TC_ORDER_DEGREE = 0
TC_ORDER_ID = 1

TC_PROBE_AUTO = 0
TC_PROBE_SORTED = 1


class TcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


class tc_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("offset_bytes", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class tc_tune(ctypes.Structure):
    _fields_ = [("small_max", ctypes.c_int32), ("probe", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("max_kicks", ctypes.c_int32),
                ("split_log2", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"small_max": self.small_max, "probe": self.probe,
                "blocks_per_cu": self.blocks_per_cu, "max_kicks": self.max_kicks,
                "split_log2": self.split_log2}


def make_tune(small_max: int = 0, probe: int = TC_PROBE_AUTO, blocks_per_cu: int = 0,
              max_kicks: int = 0, split_log2: int = 0) -> tc_tune:
    return tc_tune(small_max, probe, blocks_per_cu, max_kicks, split_log2)


def _tune_ref(tune):
    if tune is None:
        return None
    if isinstance(tune, dict):
        tune = make_tune(**tune)
    return ctypes.byref(tune)


def _load() -> ctypes.CDLL:
    if not _LIB_PATH.exists():
        raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -m paper_1909_02127_amd.build)")
    lib = ctypes.CDLL(str(_LIB_PATH))
    i64, i32, p, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)
    csr = ctypes.POINTER(tc_csr)
    lib.tc_build_csr.restype = i32
    lib.tc_build_csr.argtypes = [i64, i64, p, p, i32, p, p, i64, p, p, sz, p]
    lib.tc_orient.restype = i32
    lib.tc_orient.argtypes = [csr, i32, p, p, i64, p, p, sz, p]
    tune = ctypes.POINTER(tc_tune)
    lib.tc_count.restype = i32
    lib.tc_count.argtypes = [csr, p, tune, p, sz, p]
    lib.tc_count_per_vertex.restype = i32
    lib.tc_count_per_vertex.argtypes = [csr, p, p, tune, p, sz, p]
    lib.tc_count_per_vertex_noalloc.restype = i32
    lib.tc_count_per_vertex_noalloc.argtypes = [csr, p, p, tune, p]
    lib.tc_count_batched.restype = i32
    lib.tc_count_batched.argtypes = [csr, i64, p, p, p, p, tune, p, sz, p]
    lib.tc_pack_pairs.restype = i32
    lib.tc_pack_pairs.argtypes = [i64, p, p, p, p, p]
    lib.tc_count_k4.restype = i32
    lib.tc_count_k4.argtypes = [csr, p, p, sz, p]
    lib.tc_ne_filter.restype = i32
    lib.tc_ne_filter.argtypes = [csr, i32, i32, p, p, p, sz, p]
    lib.tc_count_bfs.restype = i32
    lib.tc_count_bfs.argtypes = [csr, p, i64, p, i64, p, p, p, sz, p]
    lib.tc_edge_support.restype = i32
    lib.tc_edge_support.argtypes = [csr, p, i64, p, p, tune, p, sz, p]
    lib.tc_source_work.restype = i32
    lib.tc_source_work.argtypes = [csr, p, p, p, sz, p]
    lib.tc_segmented_intersect.restype = i32
    lib.tc_segmented_intersect.argtypes = [csr, i64, p, p, p, p, sz, p]
    lib.tc_count_diamonds.restype = i32
    lib.tc_count_diamonds.argtypes = [csr, i64, p, p, tune, p, sz, p]
    lib.tc_count_labelled.restype = i32
    lib.tc_count_labelled.argtypes = [csr, i64, p, i32, i32, i32, p, p, tune, p, sz, p]
    lib.tc_edge_directions.restype = i32
    lib.tc_edge_directions.argtypes = [csr, i64, i64, p, p, p, p, p]
    lib.tc_count_directed.restype = i32
    lib.tc_count_directed.argtypes = [csr, p, i32, i32, i32, i32, p, tune, p, sz, p]
    lib.tc_edge_labels.restype = i32
    lib.tc_edge_labels.argtypes = [csr, i64, i64, p, p, p, p, p, p]
    lib.tc_count_edge_labelled.restype = i32
    lib.tc_count_edge_labelled.argtypes = [csr, i64, p, i32, i32, i32, p, p, tune, p, sz, p]
    lib.tc_list_triangles.restype = i32
    lib.tc_list_triangles.argtypes = [csr, p, i64, p, tune, p, sz, p]
    lib.tc_status_string.restype = ctypes.c_char_p
    lib.tc_status_string.argtypes = [i32]
    lib.tc_last_error.restype = ctypes.c_char_p
    lib.tc_last_error.argtypes = []
    lib.tc_version.restype = i32
    lib.tc_version.argtypes = []
    return lib


LIB = _load()
LIB_PATH = str(_LIB_PATH)


def status_string(status: int) -> str:
    return LIB.tc_status_string(status).decode()


def _check(status: int) -> None:
    if status != TC_OK:
        raise TcError(status, LIB.tc_last_error().decode())


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to libtc must be contiguous")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else None


def _stream(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_csr(n: int, row_ptr: torch.Tensor, col: torch.Tensor) -> tc_csr:
    if row_ptr.dtype not in (torch.int32, torch.int64) or col.dtype != torch.int32:
        raise ValueError("row_ptr must be int32/int64 and col int32")
    return tc_csr(n, row_ptr.element_size(), _ptr(row_ptr), _ptr(col))


def _ws_query(fn, *args) -> int:
    size = ctypes.c_size_t(0)
    _check(fn(*args, None, ctypes.byref(size), None))
    return int(size.value)


def _ws_call(fn, ws: torch.Tensor, *args, stream=None) -> None:
    size = ctypes.c_size_t(ws.numel() * ws.element_size())
    _check(fn(*args, _ptr(ws), ctypes.byref(size), _stream(stream)))


# ---- the C ABI, one function each ---------------------------------------------

def tc_build_csr_workspace(n: int, num_pairs: int, offset_bytes: int = 4) -> int:
    return _ws_query(LIB.tc_build_csr, n, num_pairs, None, None, offset_bytes, None, None, 0, None)


def tc_build_csr(n: int, src: torch.Tensor, dst: torch.Tensor, row_ptr: torch.Tensor,
                 col: torch.Tensor, nnz_out: torch.Tensor, ws: torch.Tensor, *, stream=None) -> None:
    if src.dtype != torch.int32 or dst.dtype != torch.int32 or src.numel() != dst.numel():
        raise ValueError("src and dst must be int32 tensors of equal length")
    if nnz_out.dtype != torch.int64 or row_ptr.numel() != n + 1:
        raise ValueError("nnz_out must be int64[1] and row_ptr must hold n+1 offsets")
    _ws_call(LIB.tc_build_csr, ws, n, src.numel(), _ptr(src), _ptr(dst), row_ptr.element_size(),
             _ptr(row_ptr), _ptr(col), col.numel(), _ptr(nnz_out), stream=stream)


def tc_orient_workspace(n: int, dag_col_capacity: int) -> int:
    """Workspace bytes of tc_orient for n vertices and a DAG column capacity (the
    workspace holds per-tile state for up to 2 * dag_col_capacity symmetric entries)."""
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_orient, ctypes.byref(csr), TC_ORDER_DEGREE, None, None,
                     dag_col_capacity, None)


def tc_orient(n: int, row_ptr: torch.Tensor, col: torch.Tensor, order: int,
              dag_row_ptr: torch.Tensor, dag_col: torch.Tensor, m_out: torch.Tensor,
              ws: torch.Tensor, *, stream=None) -> None:
    if dag_row_ptr.dtype != row_ptr.dtype or dag_row_ptr.numel() != n + 1:
        raise ValueError("dag_row_ptr must match row_ptr's dtype and hold n+1 offsets")
    csr = make_csr(n, row_ptr, col)
    _ws_call(LIB.tc_orient, ws, ctypes.byref(csr), order, _ptr(dag_row_ptr), _ptr(dag_col),
             dag_col.numel(), _ptr(m_out), stream=stream)


def tc_count_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_count, ctypes.byref(csr), None, None)


def tc_count(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor, total: torch.Tensor,
             ws: torch.Tensor, *, tune=None, stream=None) -> None:
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count, ws, ctypes.byref(csr), _ptr(total), _tune_ref(tune), stream=stream)


def tc_count_per_vertex_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_count_per_vertex, ctypes.byref(csr), None, None, None)


def tc_count_per_vertex(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                        per_vertex: torch.Tensor, total: torch.Tensor | None, ws: torch.Tensor, *,
                        tune=None, stream=None) -> None:
    if per_vertex.numel() != n:
        raise ValueError("per_vertex must hold n counts")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_per_vertex, ws, ctypes.byref(csr), _ptr(per_vertex), _ptr(total),
             _tune_ref(tune), stream=stream)


def tc_count_per_vertex_noalloc(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                                per_vertex: torch.Tensor, total: torch.Tensor | None, *,
                                tune=None, stream=None) -> None:
    """tc_count_per_vertex with its scratch in the library's static device array (no
    workspace argument; n up to 2^22)."""
    if per_vertex.numel() != n:
        raise ValueError("per_vertex must hold n counts")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _check(LIB.tc_count_per_vertex_noalloc(ctypes.byref(csr), _ptr(per_vertex), _ptr(total),
                                           _tune_ref(tune), _stream(stream)))


def tc_count_batched_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_count_batched, ctypes.byref(csr), 0, None, None, None, None, None)


def tc_count_batched(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                     vtx_off: torch.Tensor, totals: torch.Tensor, ws: torch.Tensor, *,
                     per_vertex: torch.Tensor | None = None, total: torch.Tensor | None = None,
                     tune=None, stream=None) -> None:
    g = vtx_off.numel() - 1
    if vtx_off.dtype != torch.int64 or g < 0 or totals.numel() != g:
        raise ValueError("vtx_off must be int64[G+1] and totals must hold G counts")
    if per_vertex is not None and per_vertex.numel() != n:
        raise ValueError("per_vertex must hold n counts")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_batched, ws, ctypes.byref(csr), g, _ptr(vtx_off), _ptr(totals),
             _ptr(per_vertex), _ptr(total), _tune_ref(tune), stream=stream)


def tc_pack_pairs(pair_off: torch.Tensor, vtx_off: torch.Tensor, src: torch.Tensor,
                  dst: torch.Tensor, *, stream=None) -> None:
    """In place: graph g's pairs src/dst[pair_off[g]:pair_off[g+1]] move from local ids to
    vtx_off[g] + id (ids outside the graph become -1)."""
    g = pair_off.numel() - 1
    if pair_off.dtype != torch.int64 or vtx_off.dtype != torch.int64 or vtx_off.numel() != g + 1:
        raise ValueError("pair_off and vtx_off must be int64[G+1]")
    if src.dtype != torch.int32 or dst.dtype != torch.int32 or src.numel() != dst.numel():
        raise ValueError("src and dst must be int32 tensors of equal length")
    _check(LIB.tc_pack_pairs(max(g, 0), _ptr(pair_off), _ptr(vtx_off), _ptr(src), _ptr(dst),
                             _stream(stream)))


def tc_count_k4_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_count_k4, ctypes.byref(csr), None)


def tc_count_k4(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor, total: torch.Tensor,
                ws: torch.Tensor, *, stream=None) -> None:
    """4-cliques of the oriented graph into total (int64[1], read as uint64)."""
    if total.dtype != torch.int64 or total.numel() != 1:
        raise ValueError("total must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_k4, ws, ctypes.byref(csr), _ptr(total), stream=stream)


def tc_ne_filter_workspace(n: int, max_rounds: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_ne_filter, ctypes.byref(csr), 2, max_rounds, None, None)


def tc_ne_filter(n: int, row_ptr: torch.Tensor, col: torch.Tensor, keep: torch.Tensor,
                 stats: torch.Tensor, ws: torch.Tensor, *, min_degree: int = 2,
                 max_rounds: int = 64, stream=None) -> None:
    """keep (uint8[n]) receives the candidates left by max_rounds rounds of the NE filter;
    stats (int64[3]) = kept, rounds that removed something, converged."""
    if keep.dtype != torch.uint8 or keep.numel() < n or stats.dtype != torch.int64 \
            or stats.numel() < 3:
        raise ValueError("keep must be uint8[n] and stats int64[3]")
    csr = make_csr(n, row_ptr, col)
    _ws_call(LIB.tc_ne_filter, ws, ctypes.byref(csr), min_degree, max_rounds, _ptr(keep),
             _ptr(stats), stream=stream)


def tc_count_bfs_workspace(n: int, frontier_capacity: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_count_bfs, ctypes.byref(csr), None, frontier_capacity, None, 0,
                     None, None)


def tc_count_bfs(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor, stats: torch.Tensor,
                 ws: torch.Tensor, *, frontier_capacity: int, keep: torch.Tensor | None = None,
                 matches: torch.Tensor | None = None, total: torch.Tensor | None = None,
                 stream=None) -> None:
    """The two-iteration advance; stats (int64[4]) = frontier, candidate wedges, matches,
    status; matches (int32[capacity, 3]) optional."""
    if stats.dtype != torch.int64 or stats.numel() < 4:
        raise ValueError("stats must be int64[4]")
    if matches is not None and (matches.dtype != torch.int32 or matches.dim() != 2
                                or matches.shape[1] != 3):
        raise ValueError("matches must be int32 of shape (capacity, 3)")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_bfs, ws, ctypes.byref(csr), _ptr(keep), frontier_capacity,
             _ptr(matches), 0 if matches is None else matches.shape[0], _ptr(stats), _ptr(total),
             stream=stream)


def tc_edge_support_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_edge_support, ctypes.byref(csr), None, 0, None, None, None)


def tc_edge_support(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                    support: torch.Tensor, m_out: torch.Tensor, ws: torch.Tensor, *,
                    total: torch.Tensor | None = None, tune=None, stream=None) -> None:
    """support (int32 or uint32 storage, capacity entries) receives the triangles on each
    oriented edge; m_out (int64[1]) receives m or -TC_ERR_CAPACITY."""
    if support.element_size() != 4 or m_out.dtype != torch.int64 or m_out.numel() != 1:
        raise ValueError("support must hold 4-byte counts and m_out must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_edge_support, ws, ctypes.byref(csr), _ptr(support), support.numel(),
             _ptr(m_out), _ptr(total), _tune_ref(tune), stream=stream)


def tc_source_work_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_source_work, ctypes.byref(csr), None, None)


def tc_source_work(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                   prefix: torch.Tensor, ws: torch.Tensor, *, work: torch.Tensor | None = None,
                   stream=None) -> None:
    """w(u) (int64[n], optional) and its exclusive prefix (int64[n+1]) of a DAG."""
    if prefix.dtype != torch.int64 or prefix.numel() != n + 1:
        raise ValueError("prefix must be int64[n+1]")
    if work is not None and (work.dtype != torch.int64 or work.numel() != n):
        raise ValueError("work must be int64[n]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_source_work, ws, ctypes.byref(csr), _ptr(work), _ptr(prefix), stream=stream)


def tc_segmented_intersect_workspace(n: int, edge_capacity: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_segmented_intersect, ctypes.byref(csr), edge_capacity, None, None,
                     None)


def tc_segmented_intersect(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                           total: torch.Tensor, m_out: torch.Tensor, ws: torch.Tensor, *,
                           support: torch.Tensor | None = None, stream=None) -> None:
    """Merge-path intersection of N+(u) and N+(v) for every DAG edge: total (int64[1])
    receives T; with support (4-byte counts, at least dag_col.numel() entries) every
    edge's triangles; m_out (int64[1]) receives m or -TC_ERR_CAPACITY.  The edge capacity
    is dag_col.numel()."""
    if m_out.dtype != torch.int64 or m_out.numel() != 1:
        raise ValueError("m_out must be int64[1]")
    cap = dag_col.numel()
    if support is not None and (support.element_size() != 4 or support.numel() < cap):
        raise ValueError("support must hold 4-byte counts for every dag_col entry")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_segmented_intersect, ws, ctypes.byref(csr), cap, _ptr(total),
             _ptr(support), _ptr(m_out), stream=stream)


def tc_count_diamonds_workspace(n: int, edge_capacity: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_count_diamonds, ctypes.byref(csr), edge_capacity, None, None, None)


def tc_count_diamonds(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                      total: torch.Tensor, m_out: torch.Tensor, ws: torch.Tensor, *, tune=None,
                      stream=None) -> None:
    """Number of diamonds (two triangles sharing an edge) into total (int64[1]); m_out
    (int64[1]) receives m or -TC_ERR_CAPACITY.  The edge capacity is dag_col.numel()."""
    if m_out.dtype != torch.int64 or m_out.numel() != 1:
        raise ValueError("m_out must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_diamonds, ws, ctypes.byref(csr), dag_col.numel(), _ptr(total),
             _ptr(m_out), _tune_ref(tune), stream=stream)


def tc_count_labelled_workspace(n: int, edge_capacity: int, offset_bytes: int = 4) -> int:
    csr = tc_csr(n, offset_bytes, None, None)
    return _ws_query(LIB.tc_count_labelled, ctypes.byref(csr), edge_capacity, None, 0, 0, 0, None,
                     None, None)


def tc_count_labelled(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                      labels: torch.Tensor, query, total: torch.Tensor, ws: torch.Tensor, *,
                      kept_out: torch.Tensor | None = None, tune=None, stream=None) -> None:
    """Triangles whose vertex labels equal the query's three labels (as a multiset) into
    total (int64[1]); kept_out (int64[1]) receives the DAG edges whose labels fit the
    query, or -TC_ERR_CAPACITY.  The edge capacity is dag_col.numel()."""
    if labels.dtype != torch.int32 or labels.numel() < n:
        raise ValueError("labels must be int32 with one entry per vertex")
    q = [int(x) for x in query]
    if len(q) != 3:
        raise ValueError("the query has three labels")
    if kept_out is not None and (kept_out.dtype != torch.int64 or kept_out.numel() != 1):
        raise ValueError("kept_out must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_labelled, ws, ctypes.byref(csr), dag_col.numel(), _ptr(labels), *q,
             _ptr(total), _ptr(kept_out), _tune_ref(tune), stream=stream)


def tc_edge_directions(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                       src: torch.Tensor, dst: torch.Tensor, direction: torch.Tensor,
                       m_out: torch.Tensor, *, stream=None) -> None:
    """Arc directions of the pairs src[i] -> dst[i] on the DAG built from them: direction
    (uint8, at least dag_col.numel() rounded up to 4 entries, 4-byte aligned) gets bit 0 for
    the arc from the row's vertex to the column, bit 1 for the reverse.  m_out (int64[1])
    receives m or a negative status.  The edge capacity is dag_col.numel()."""
    if src.dtype != torch.int32 or dst.dtype != torch.int32 or src.numel() != dst.numel():
        raise ValueError("src and dst must be int32 tensors of equal length")
    cap = dag_col.numel()
    if direction.dtype != torch.uint8 or direction.numel() < (cap + 3) // 4 * 4:
        raise ValueError("direction must be uint8 with dag_col.numel() rounded up to 4 entries")
    if m_out.dtype != torch.int64 or m_out.numel() != 1:
        raise ValueError("m_out must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _check(LIB.tc_edge_directions(ctypes.byref(csr), cap, src.numel(), _ptr(src), _ptr(dst),
                                  _ptr(direction), _ptr(m_out), _stream(stream)))


def tc_count_directed_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_count_directed, ctypes.byref(csr), None, 1, 1, 1, 0, None, None)


def tc_count_directed(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                      direction: torch.Tensor, pattern, total: torch.Tensor, ws: torch.Tensor, *,
                      induced: bool = False, tune=None, stream=None) -> None:
    """Matches of the directed triangle query pattern = (p01, p02, p12) (each 1: lower ->
    higher node, 2: the reverse, 3: both) into total (int64[1]), on the DAG and the arc
    directions tc_edge_directions wrote for it."""
    p = [int(x) for x in pattern]
    if len(p) != 3:
        raise ValueError("the pattern has three node pairs")
    if direction.dtype != torch.uint8 or direction.numel() < dag_col.numel():
        raise ValueError("direction must be uint8 with one entry per dag_col entry")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_directed, ws, ctypes.byref(csr), _ptr(direction), *p,
             int(bool(induced)), _ptr(total), _tune_ref(tune), stream=stream)


def tc_edge_labels(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                   src: torch.Tensor, dst: torch.Tensor, labels: torch.Tensor,
                   edge_labels: torch.Tensor, m_out: torch.Tensor, *, stream=None) -> None:
    """Labels (uint8, 0..3) of the pairs {src[i], dst[i]} on the DAG built from them:
    edge_labels (uint8, at least dag_col.numel() rounded up to 4 entries) gets each edge's
    largest label; m_out (int64[1]) receives m or a negative status.  The edge capacity is
    dag_col.numel()."""
    if src.dtype != torch.int32 or dst.dtype != torch.int32 or src.numel() != dst.numel():
        raise ValueError("src and dst must be int32 tensors of equal length")
    if labels.dtype != torch.uint8 or labels.numel() != src.numel():
        raise ValueError("labels must be uint8 with one entry per pair")
    cap = dag_col.numel()
    if edge_labels.dtype != torch.uint8 or edge_labels.numel() < (cap + 3) // 4 * 4:
        raise ValueError("edge_labels must be uint8 with dag_col.numel() rounded up to 4 entries")
    if m_out.dtype != torch.int64 or m_out.numel() != 1:
        raise ValueError("m_out must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _check(LIB.tc_edge_labels(ctypes.byref(csr), cap, src.numel(), _ptr(src), _ptr(dst),
                              _ptr(labels), _ptr(edge_labels), _ptr(m_out), _stream(stream)))


def tc_count_edge_labelled_workspace(n: int, edge_capacity: int, offset_bytes: int = 4) -> int:
    csr = tc_csr(n, offset_bytes, None, None)
    return _ws_query(LIB.tc_count_edge_labelled, ctypes.byref(csr), edge_capacity, None, 0, 0, 0,
                     None, None, None)


def tc_count_edge_labelled(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                           edge_labels: torch.Tensor, query, total: torch.Tensor,
                           ws: torch.Tensor, *, kept_out: torch.Tensor | None = None, tune=None,
                           stream=None) -> None:
    """Triangles whose edges carry the query's labels (q01, q02, q12) into total (int64[1]),
    on the DAG and the labels tc_edge_labels wrote for it; kept_out (int64[1]) receives the
    DAG edges whose label is in the query, or -TC_ERR_CAPACITY.  The edge capacity is
    dag_col.numel()."""
    q = [int(x) for x in query]
    if len(q) != 3:
        raise ValueError("the query has three edges")
    if edge_labels.dtype != torch.uint8 or edge_labels.numel() < dag_col.numel():
        raise ValueError("edge_labels must be uint8 with one entry per dag_col entry")
    if kept_out is not None and (kept_out.dtype != torch.int64 or kept_out.numel() != 1):
        raise ValueError("kept_out must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_count_edge_labelled, ws, ctypes.byref(csr), dag_col.numel(), _ptr(edge_labels),
             *q, _ptr(total), _ptr(kept_out), _tune_ref(tune), stream=stream)


def tc_list_triangles_workspace(n: int) -> int:
    csr = tc_csr(n, 4, None, None)
    return _ws_query(LIB.tc_list_triangles, ctypes.byref(csr), None, 0, None, None)


def tc_list_triangles(n: int, dag_row_ptr: torch.Tensor, dag_col: torch.Tensor,
                      triples: torch.Tensor, count_out: torch.Tensor, ws: torch.Tensor, *,
                      tune=None, stream=None) -> None:
    """Rows (u, v, w) of every triangle into triples (int32[capacity, 3]); count_out
    (int64[1]) receives T or -TC_ERR_CAPACITY."""
    if triples.dtype != torch.int32 or triples.dim() != 2 or triples.shape[1] != 3:
        raise ValueError("triples must be an int32 tensor of shape (capacity, 3)")
    if count_out.dtype != torch.int64 or count_out.numel() != 1:
        raise ValueError("count_out must be int64[1]")
    csr = make_csr(n, dag_row_ptr, dag_col)
    _ws_call(LIB.tc_list_triangles, ws, ctypes.byref(csr), _ptr(triples), triples.shape[0],
             _ptr(count_out), _tune_ref(tune), stream=stream)


def tc_version() -> int:
    return int(LIB.tc_version())
