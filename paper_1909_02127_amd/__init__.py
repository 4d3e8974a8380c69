"""MI355X-native exact triangle counting (Wang & Owens, "Fast BFS-Based Triangle
Counting on GPUs"): a C ABI library of hand-written gfx950 HIP kernels
(libtc.so) and a thin Python binding over it.

    from paper_1909_02127_amd import triangle_count
    res = triangle_count(src, dst, n, per_vertex=True)   # src/dst: int32 CUDA tensors

Importing the package requires the built library; there is no CPU fallback.
"""
from ._lib import (TC_ORDER_DEGREE, TC_ORDER_ID, TC_PROBE_AUTO, TC_PROBE_SORTED,  # noqa: F401
                   TcError, make_tune, tc_build_csr, tc_count, tc_count_batched,
                   tc_count_per_vertex, tc_orient, tc_version)
from .pipeline import Pipeline, Result, triangle_count  # noqa: F401
