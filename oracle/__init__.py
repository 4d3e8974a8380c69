"""CPU oracle for exact triangle counting (ctypes wrapper over ``tc_oracle.c``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The library's product
path never calls it, and it imports nothing from the product package.

Each function follows a definition of Wang & Owens, "Fast BFS-Based Triangle
Counting on GPUs" (problem definition Sec. II-A, Def. 1-2; Alg. 1 unique mapping
order and non-tree-edge check); the C source states which one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "tc_oracle.c"
_LIB = _HERE / "liboracle.so"

ORDER_DEGREE = 0
ORDER_ID = 1
ORDER_KEY = 2


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (plain C99 + OpenMP, no target-specific flags)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", str(_SRC),
                        "-o", str(tmp)], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build(force=True)
        lib = ctypes.CDLL(str(_LIB))
        i64, i32, p = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.oracle_clean.restype = i64
        lib.oracle_clean.argtypes = [i64, i64, p, p, p, p, i64]
        lib.oracle_orient.restype = i64
        lib.oracle_orient.argtypes = [i64, p, p, i32, p, p, p]
        lib.oracle_count.restype = ctypes.c_uint64
        lib.oracle_count.argtypes = [i64, i64, p, p, p, i32]
        lib.oracle_vertex_triangles.restype = i64
        lib.oracle_vertex_triangles.argtypes = [i64, i64, p, p, i32]
        lib.oracle_count_k4.restype = ctypes.c_uint64
        lib.oracle_count_k4.argtypes = [i64, p, p]
        lib.oracle_count_diamonds.restype = ctypes.c_uint64
        lib.oracle_count_diamonds.argtypes = [i64, i64, p, p]
        lib.oracle_count_labelled.restype = ctypes.c_uint64
        lib.oracle_count_labelled.argtypes = [i64, p, p, p, i32, i32, i32]
        lib.oracle_count_edge_labelled.restype = i64
        lib.oracle_count_edge_labelled.argtypes = [i64, p, p, i64, p, p, p, i32, i32, i32, i64]
        lib.oracle_count_directed.restype = i64
        lib.oracle_count_directed.argtypes = [i64, p, p, i64, p, p, i32, i32, i32, i32, i64]
        lib.oracle_kcore.restype = i64
        lib.oracle_kcore.argtypes = [i64, p, p, i32, p]
        lib.oracle_edge_support.restype = i64
        lib.oracle_edge_support.argtypes = [i64, p, p, p]
        lib.oracle_list.restype = i64
        lib.oracle_list.argtypes = [i64, p, p, p, i64]
        lib.oracle_max_threads.restype = i32
        lib.oracle_max_threads.argtypes = []
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


class OracleError(ValueError):
    pass


def clean(n: int, src, dst) -> tuple[np.ndarray, np.ndarray]:
    """Raw pairs -> symmetric deduplicated self-loop-free CSR (row_ptr int64, col int32)."""
    lib = _load()
    src, dst = _i32(src), _i32(dst)
    if src.shape != dst.shape:
        raise OracleError("src and dst differ in length")
    p = src.size
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(2 * p, 1), dtype=np.int32)
    nnz = lib.oracle_clean(n, p, _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col), col.size)
    if nnz == -2:
        raise OracleError("vertex id outside [0, n)")
    if nnz < 0:
        raise OracleError(f"oracle_clean failed ({nnz})")
    return row_ptr, col[:nnz].copy()


def orient(row_ptr: np.ndarray, col: np.ndarray, order: int = ORDER_DEGREE,
           key: np.ndarray | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Keep (u, v) iff rank(u) < rank(v); rank = (degree, id), id, or (key, id)."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = _i32(col)
    n = row_ptr.size - 1
    if order == ORDER_KEY:
        if key is None or key.size != n:
            raise OracleError("ORDER_KEY needs a key per vertex")
        key = np.ascontiguousarray(key, dtype=np.int64)
    else:
        key = None
    dag_ptr = np.zeros(n + 1, dtype=np.int64)
    dag_col = np.zeros(max(col.size // 2, 1), dtype=np.int32)
    m = lib.oracle_orient(n, _ptr(row_ptr), _ptr(col), order, _ptr(key), _ptr(dag_ptr),
                          _ptr(dag_col))
    return dag_ptr, dag_col[:m].copy()


def count(dag_ptr: np.ndarray, dag_col: np.ndarray, *, per_vertex: bool = False,
          threads: int = 0, sources=None):
    """Triangles of an oriented graph; with per_vertex, also t(v) as uint64[n].  With
    `sources`, only the triangles whose source u (lowest rank) has an id below it."""
    lib = _load()
    dag_ptr = np.ascontiguousarray(dag_ptr, dtype=np.int64)
    dag_col = _i32(dag_col)
    n = dag_ptr.size - 1
    t = np.zeros(max(n, 1), dtype=np.uint64) if per_vertex else None
    total = int(lib.oracle_count(n, _sources(dag_ptr, sources), _ptr(dag_ptr), _ptr(dag_col),
                                 _ptr(t), threads))
    if per_vertex:
        return total, t[:n].copy()
    return total


def _sources(dag_ptr: np.ndarray, sources) -> int:
    """Sources to enumerate: all n, or the first `sources` ids (a timing sample;
    the rows of every vertex stay readable)."""
    n = dag_ptr.size - 1
    return n if sources is None else max(0, min(int(sources), n))


def list_triangles(dag_ptr: np.ndarray, dag_col: np.ndarray, sources=None) -> np.ndarray:
    """The triangles of an oriented graph as an int32 array of shape (T, 3): rows
    (u, v, w) with v, w in N+(u) and w in N+(v), in lexicographic order.  With
    `sources`, only the triangles whose source u (lowest rank) has an id below it."""
    lib = _load()
    dag_ptr = np.ascontiguousarray(dag_ptr, dtype=np.int64)
    dag_col = _i32(dag_col)
    n = _sources(dag_ptr, sources)
    total = int(lib.oracle_list(n, _ptr(dag_ptr), _ptr(dag_col), None, 0))
    out = np.zeros((max(total, 1), 3), dtype=np.int32)
    got = int(lib.oracle_list(n, _ptr(dag_ptr), _ptr(dag_col), _ptr(out), total))
    if got != total:
        raise OracleError("oracle_list changed its answer")
    return out[:total].copy()


def count_k4(dag_ptr: np.ndarray, dag_col: np.ndarray, sources=None) -> int:
    """Number of 4-cliques of an oriented graph (each found once).  With `sources`,
    only those whose source (lowest rank) has an id below it."""
    lib = _load()
    dag_ptr = np.ascontiguousarray(dag_ptr, dtype=np.int64)
    dag_col = _i32(dag_col)
    r = int(lib.oracle_count_k4(_sources(dag_ptr, sources), _ptr(dag_ptr), _ptr(dag_col)))
    if r == (1 << 64) - 1:
        raise OracleError("oracle_count_k4: allocation failed")
    return r


def k4(n: int, src, dst, *, order: int = ORDER_DEGREE) -> int:
    """4-cliques from raw pairs: clean -> orient -> count."""
    row_ptr, col = clean(n, src, dst)
    dag_ptr, dag_col = orient(row_ptr, col, order)
    return count_k4(dag_ptr, dag_col)


def count_diamonds(row_ptr: np.ndarray, col: np.ndarray, sources=None) -> int:
    """Number of diamonds (two triangles sharing an edge, counted as subgraphs) of a
    symmetric CSR.  With `sources`, only the shared edges {b, c} (b < c) whose lower
    end b has an id below it count."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = _i32(col)
    n = row_ptr.size - 1
    lim = n if sources is None else max(0, min(int(sources), n))
    return int(lib.oracle_count_diamonds(n, lim, _ptr(row_ptr), _ptr(col)))


def diamonds(n: int, src, dst) -> int:
    """Diamonds from raw pairs: clean -> count."""
    row_ptr, col = clean(n, src, dst)
    return count_diamonds(row_ptr, col)


def count_labelled(dag_ptr: np.ndarray, dag_col: np.ndarray, labels, query) -> int:
    """Triangles of an oriented graph whose vertices' label multiset equals the query's
    three labels."""
    lib = _load()
    dag_ptr = np.ascontiguousarray(dag_ptr, dtype=np.int64)
    dag_col = _i32(dag_col)
    labels = _i32(labels)
    q = [int(x) for x in query]
    if len(q) != 3:
        raise ValueError("the query has three node labels")
    return int(lib.oracle_count_labelled(dag_ptr.size - 1, _ptr(dag_ptr), _ptr(dag_col),
                                         _ptr(labels), q[0], q[1], q[2]))


def labelled(n: int, src, dst, labels, query, *, order: int = ORDER_DEGREE) -> int:
    """Labelled triangles of a raw pair list (clean, orient, count)."""
    rp, col = clean(n, src, dst)
    dp, dc = orient(rp, col, order)
    return count_labelled(dp, dc, labels, query)


def count_directed(dag_ptr: np.ndarray, dag_col: np.ndarray, src, dst, pattern, *,
                   induced: bool = False, sources=None) -> int:
    """Matches of a directed triangle query in the arcs src[i] -> dst[i], whose underlying
    undirected graph the DAG orients.  pattern = (p01, p02, p12): for each pair of query
    nodes, bit 1 = the lower has an arc to the higher, bit 2 = the reverse.  With
    `sources`, only the triangles whose DAG source has an id below it count."""
    lib = _load()
    dag_ptr = np.ascontiguousarray(dag_ptr, dtype=np.int64)
    dag_col = _i32(dag_col)
    s, d = _i32(src), _i32(dst)
    if s.size != d.size:
        raise ValueError("src and dst differ in length")
    p = [int(x) for x in pattern]
    if len(p) != 3:
        raise ValueError("the pattern has three node pairs")
    r = int(lib.oracle_count_directed(dag_ptr.size - 1, _ptr(dag_ptr), _ptr(dag_col), s.size,
                                      _ptr(s), _ptr(d), p[0], p[1], p[2], int(bool(induced)),
                                      _sources(dag_ptr, sources)))
    if r < 0:
        raise OracleError(f"oracle_count_directed failed ({r})")
    return r


def directed(n: int, src, dst, pattern, *, induced: bool = False,
             order: int = ORDER_DEGREE) -> int:
    """Directed triangle query on a raw arc list (clean, orient, match)."""
    rp, col = clean(n, src, dst)
    dp, dc = orient(rp, col, order)
    return count_directed(dp, dc, src, dst, pattern, induced=induced)


def count_edge_labelled(dag_ptr: np.ndarray, dag_col: np.ndarray, src, dst, labels,
                        query, sources=None) -> int:
    """Triangles whose edges carry the query's edge labels (q01, q02, q12), matched as
    subgraphs; pair i has label labels[i], an edge given several times the largest.  With
    `sources`, only the triangles whose DAG source has an id below it count."""
    lib = _load()
    dag_ptr = np.ascontiguousarray(dag_ptr, dtype=np.int64)
    dag_col = _i32(dag_col)
    s, d, lab = _i32(src), _i32(dst), _i32(labels)
    if not s.size == d.size == lab.size:
        raise ValueError("src, dst and labels differ in length")
    q = [int(x) for x in query]
    if len(q) != 3:
        raise ValueError("the query has three edges")
    r = int(lib.oracle_count_edge_labelled(dag_ptr.size - 1, _ptr(dag_ptr), _ptr(dag_col), s.size,
                                           _ptr(s), _ptr(d), _ptr(lab), q[0], q[1], q[2],
                                           _sources(dag_ptr, sources)))
    if r < 0:
        raise OracleError(f"oracle_count_edge_labelled failed ({r})")
    return r


def edge_labelled(n: int, src, dst, labels, query, *, order: int = ORDER_DEGREE) -> int:
    """Edge-labelled triangle query on a raw labelled pair list (clean, orient, match)."""
    rp, col = clean(n, src, dst)
    dp, dc = orient(rp, col, order)
    return count_edge_labelled(dp, dc, src, dst, labels, query)


def kcore(row_ptr: np.ndarray, col: np.ndarray, k: int = 2) -> np.ndarray:
    """uint8[n]: 1 for the vertices of the k-core of a symmetric CSR."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = _i32(col)
    n = row_ptr.size - 1
    keep = np.zeros(max(n, 1), dtype=np.uint8)
    if lib.oracle_kcore(n, _ptr(row_ptr), _ptr(col), int(k), _ptr(keep)) < 0:
        raise OracleError("oracle_kcore failed")
    return keep[:n].copy()


def edge_support(dag_ptr: np.ndarray, dag_col: np.ndarray, sources=None) -> tuple[int, np.ndarray]:
    """(T, sup) where sup[e] (uint32, one per oriented edge) counts the triangles on edge e.
    With `sources`, only the triangles whose source (lowest rank) has an id below it count."""
    lib = _load()
    dag_ptr = np.ascontiguousarray(dag_ptr, dtype=np.int64)
    dag_col = _i32(dag_col)
    n = _sources(dag_ptr, sources)
    sup = np.zeros(max(int(dag_ptr[-1]), 1), dtype=np.uint32)
    total = int(lib.oracle_edge_support(n, _ptr(dag_ptr), _ptr(dag_col), _ptr(sup)))
    return total, sup[: int(dag_ptr[-1])].copy()


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def vertex_triangles(n: int, src, dst, v: int) -> int:
    """t(v) straight from the raw pairs: distinct edges among the neighbours of v."""
    lib = _load()
    src, dst = _i32(src), _i32(dst)
    r = lib.oracle_vertex_triangles(n, src.size, _ptr(src), _ptr(dst), int(v))
    if r < 0:
        raise OracleError("oracle_vertex_triangles failed")
    return int(r)


def triangles(n: int, src, dst, *, per_vertex: bool = False, order: int = ORDER_DEGREE,
              threads: int = 0):
    """Whole pipeline from raw pairs: clean -> orient -> count."""
    row_ptr, col = clean(n, src, dst)
    dag_ptr, dag_col = orient(row_ptr, col, order)
    return count(dag_ptr, dag_col, per_vertex=per_vertex, threads=threads)
