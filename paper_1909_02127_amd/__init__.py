"""MI355X-native exact triangle counting (Wang & Owens, "Fast BFS-Based Triangle
Counting on GPUs"): a C ABI library of hand-written gfx950 HIP kernels
(libtc.so) and a thin Python binding over it.

    from paper_1909_02127_amd import triangle_count
    res = triangle_count(src, dst, n, per_vertex=True)   # src/dst: int32 CUDA tensors

The library is loaded on first use of any of the names below, so the build
module (paper_1909_02127_amd.build) imports without it; using the package
without a built libtc.so raises ImportError (there is no CPU fallback).
"""
import importlib

_EXPORTS = {
    "TC_ORDER_DEGREE": "_lib", "TC_ORDER_ID": "_lib", "TC_PROBE_AUTO": "_lib",
    "TC_PROBE_SORTED": "_lib", "TcError": "_lib", "make_tune": "_lib", "tc_build_csr": "_lib",
    "tc_count": "_lib", "tc_count_batched": "_lib", "tc_count_per_vertex": "_lib",
    "tc_count_bfs": "_lib", "tc_count_k4": "_lib", "tc_count_diamonds": "_lib",
    "tc_segmented_intersect": "_lib", "tc_source_work": "_lib", "tc_edge_support": "_lib", "tc_list_triangles": "_lib",
    "tc_ne_filter": "_lib", "tc_orient": "_lib", "tc_version": "_lib",
    "Pipeline": "pipeline", "Result": "pipeline", "triangle_count": "pipeline",
}

__all__ = sorted(_EXPORTS)


def __getattr__(name):
    if name in _EXPORTS:
        mod = importlib.import_module(f".{_EXPORTS[name]}", __name__)
        value = getattr(mod, name)
        globals()[name] = value
        return value
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
