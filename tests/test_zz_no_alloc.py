"""tc_count_per_vertex_noalloc (scratch in the library's static device array) against
tc_count_per_vertex with a caller workspace, through the C ABI, on two calls in a row
with the second graph smaller, bit-exact; plus the size limit."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu

MAX_N = 1 << 22


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_02127_amd as tc
    return tc


def _dag(tc, scale, ef, seed, ob):
    s, d, n = graphgen.rmat(scale, ef, seed, device="cuda")
    p = tc.Pipeline(n, s.numel(), offset_bytes=ob)
    p.build(s, d)
    p.orient()
    p.result()
    return p, s, d, n


def test_noalloc_equals_workspace_path_twice_then_smaller(tc):
    from paper_1909_02127_amd import _lib
    cases = [(22, 4, 5, 8), (13, 16, 6, 4)]  # n = 2^22 (the limit), then n = 2^13
    for i, (scale, ef, seed, ob) in enumerate(cases):
        _say("noalloc call", i, "scale", scale, "ef", ef, "offsets", ob)
        p, s, d, n = _dag(tc, scale, ef, seed, ob)
        assert n <= MAX_N
        want_pv = torch.zeros(n, dtype=torch.int64, device="cuda")
        want_t = torch.zeros(1, dtype=torch.int64, device="cuda")
        _lib.tc_count_per_vertex(n, p.dag_ptr, p.dag_col, want_pv, want_t, p.ws_count)
        got_pv = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        got_t = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        _lib.tc_count_per_vertex_noalloc(n, p.dag_ptr, p.dag_col, got_pv, got_t)
        # the total is optional: without it the scratch holds the total
        got_pv2 = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        _lib.tc_count_per_vertex_noalloc(n, p.dag_ptr, p.dag_col, got_pv2, None)
        torch.cuda.synchronize()
        assert int(got_t.item()) == int(want_t.item()) > 0
        assert torch.equal(got_pv, want_pv)
        assert torch.equal(got_pv2, want_pv)
        assert int(want_pv.sum().item()) == 3 * int(want_t.item())
        if scale <= 13:
            T, t = oracle.triangles(n, s.cpu().numpy(), d.cpu().numpy(), per_vertex=True)
            assert int(got_t.item()) == T
            np.testing.assert_array_equal(got_pv.cpu().numpy().astype(np.uint64), t)
        del p


def test_noalloc_rejects_graphs_above_the_limit(tc):
    from paper_1909_02127_amd import _lib
    row_ptr = torch.zeros(2, dtype=torch.int32, device="cuda")
    col = torch.zeros(1, dtype=torch.int32, device="cuda")
    pv = torch.zeros(1, dtype=torch.int64, device="cuda")
    csr = _lib.tc_csr(MAX_N + 1, 4, row_ptr.data_ptr(), col.data_ptr())
    import ctypes
    st = _lib.LIB.tc_count_per_vertex_noalloc(ctypes.byref(csr), ctypes.c_void_p(pv.data_ptr()),
                                              None, None, None)
    assert st == _lib.TC_ERR_CAPACITY
    assert "static scratch" in _lib.LIB.tc_last_error().decode()
