"""GPU check of tc_source_work: w(u) = sum of d+(v) over N+(u) (0 when d+(u) < 2) and its
exclusive prefix, against the definition written out in numpy on the oracle's DAG."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests import pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_02127_amd as tc
    return tc


def _want(n, s, d, order):
    rp, col = oracle.clean(n, np.asarray(s), np.asarray(d))
    dp, dc = oracle.orient(rp, col, order)
    dplus = np.diff(dp)
    rows = np.repeat(np.arange(n), dplus)
    w = np.bincount(rows, weights=dplus[dc], minlength=n).astype(np.int64) if n else \
        np.zeros(0, np.int64)
    w[dplus < 2] = 0
    return w, np.concatenate([[0], np.cumsum(w)]).astype(np.int64)


@pytest.mark.parametrize("ob", [4, 8])
def test_source_work_against_definition(tc, ob):
    from paper_1909_02127_amd import _lib
    cases = [pins.complete(30), pins.wheel(12), (1, [0], [0]), (0, [], [])]
    s, d, n = graphgen.rmat(14, 16, 3)
    cases.append((n, s.numpy(), d.numpy()))
    s, d, n = graphgen.erdos_renyi(1024, 8192, 2)
    cases.append((n, s.numpy(), d.numpy()))
    for n, s, d in cases:
        for order in (0, 1):
            p = tc.Pipeline(n, max(len(s), 1), offset_bytes=ob, order=order)
            p.build(torch.as_tensor(np.asarray(s, np.int32)).cuda(),
                    torch.as_tensor(np.asarray(d, np.int32)).cuda())
            p.orient()
            p.result()
            work = torch.full((n,), -1, dtype=torch.int64, device="cuda")
            prefix = torch.full((n + 1,), -1, dtype=torch.int64, device="cuda")
            ws = torch.empty(_lib.tc_source_work_workspace(n), dtype=torch.uint8, device="cuda")
            _lib.tc_source_work(n, p.dag_ptr, p.dag_col, prefix, ws, work=work)
            prefix2 = torch.full((n + 1,), -1, dtype=torch.int64, device="cuda")
            _lib.tc_source_work(n, p.dag_ptr, p.dag_col, prefix2, ws)
            torch.cuda.synchronize()
            w, pre = _want(n, s, d, order)
            np.testing.assert_array_equal(work.cpu().numpy(), w)
            np.testing.assert_array_equal(prefix.cpu().numpy(), pre)
            np.testing.assert_array_equal(prefix2.cpu().numpy(), pre)


def test_source_work_scale20_total_is_the_wedge_count(tc):
    """The benchmark graph: the prefix's last entry is W (the wedges the count enumerates),
    and cutting the sources at equal prefix sums gives 8 ranges of equal work within the
    largest single w(u)."""
    from paper_1909_02127_amd import _lib
    s, d, n = graphgen.rmat(20, 16, 20, device="cuda")
    p = tc.Pipeline(n, s.numel())
    p.build(s, d)
    p.orient()
    p.result()
    work = torch.empty(n, dtype=torch.int64, device="cuda")
    prefix = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ws = torch.empty(_lib.tc_source_work_workspace(n), dtype=torch.uint8, device="cuda")
    _lib.tc_source_work(n, p.dag_ptr, p.dag_col, prefix, ws, work=work)
    w, pre = _want(n, s.cpu().numpy(), d.cpu().numpy(), 0)
    np.testing.assert_array_equal(prefix.cpu().numpy(), pre)
    W = int(pre[-1])
    cuts = np.searchsorted(pre, [W * k // 8 for k in range(9)])
    shares = np.diff(pre[np.clip(cuts, 0, n)])
    assert abs(int(shares.max()) - W // 8) <= int(w.max())
