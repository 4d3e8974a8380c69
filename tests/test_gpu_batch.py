"""GPU parity of the batched path: per-graph totals of one packed launch sequence equal the
plain one-graph-per-launch path and the oracle, graph by graph, bit-exact."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests import pins

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_02127_amd as tc
    return tc


def _suite(count, seed, log2_min=5, log2_max=11):
    spec = graphgen.batch_suite_spec(count, seed=seed, log2_min=log2_min, log2_max=log2_max)
    return [graphgen.batch_graph(g, device="cuda") for g in spec]


def _oracle_totals(graphs):
    out, per = [], []
    for s, d, n in graphs:
        t, p = oracle.triangles(n, s.cpu().numpy(), d.cpu().numpy(), per_vertex=True)
        out.append(t)
        per.append(p)
    return out, np.concatenate(per) if per else np.zeros(0, np.uint64)


@pytest.mark.parametrize("offset_bytes", [4, 8])
def test_batched_equals_plain_equals_oracle(tc, offset_bytes):
    from paper_1909_02127_amd.batch import BatchRunner, PackedBatch, PlainRunner
    graphs = _suite(48, 41)
    _say("batch of", len(graphs))
    want, want_pv = _oracle_totals(graphs)
    b = PackedBatch(graphs, offset_bytes=offset_bytes)
    br = BatchRunner(b, per_vertex=True)
    br.enqueue()
    totals, grand = br.results()
    assert totals == want
    assert grand == sum(want)
    np.testing.assert_array_equal(br.pv[: b.n].cpu().numpy().astype(np.uint64), want_pv)
    pr = PlainRunner(b)
    pr.enqueue()
    assert pr.results() == want


def test_batched_hip_graph_replays(tc):
    """Replays interleaved with eager work each give the eager result."""
    from paper_1909_02127_amd.batch import BatchRunner, PackedBatch
    graphs = _suite(32, 7)
    b = PackedBatch(graphs)
    br = BatchRunner(b, tune={"small_max": 32})
    br.enqueue()
    eager, grand = br.results()
    br.capture()
    for k in range(4):
        br.totals.fill_(-1)
        br.total.fill_(-1)
        br.replay()
        got, g2 = br.results()
        assert got == eager and g2 == grand, f"replay {k}"
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()  # unrelated eager work between replays
    want, _ = _oracle_totals(graphs)
    assert eager == want


def test_batched_tuning_never_changes_counts(tc):
    from paper_1909_02127_amd.batch import BatchRunner, PackedBatch
    graphs = _suite(24, 99, log2_min=6, log2_max=12)
    want, _ = _oracle_totals(graphs)
    b = PackedBatch(graphs)
    for tune in [None, {"small_max": 1}, {"small_max": 16}, {"probe": tc.TC_PROBE_SORTED},
                 {"blocks_per_cu": 1}, {"small_max": 64, "probe": 1, "blocks_per_cu": 2},
                 {"small_max": 96}, {"small_max": 8, "split_log2": 3},
                 {"split_log2": -1}]:
        br = BatchRunner(b, tune=tune)
        br.enqueue()
        assert br.results()[0] == want, tune


def test_batched_edge_cases(tc):
    from paper_1909_02127_amd import _lib
    from paper_1909_02127_amd.batch import BatchRunner, PackedBatch
    z = torch.zeros(0, dtype=torch.int32)
    cases = [
        [pins.complete(5), pins.petersen(), pins.wheel(7)],
        [(3, [], []), pins.complete(4), (2, [], [])],     # graphs without edges
        [pins.friendship(6)],                              # a single graph
    ]
    for parts in cases:
        graphs = [(torch.tensor(s, dtype=torch.int32) if len(s) else z,
                   torch.tensor(d, dtype=torch.int32) if len(d) else z, n) for n, s, d in parts]
        want = [oracle.triangles(n, np.array(s, np.int32), np.array(d, np.int32)) for n, s, d in parts]
        b = PackedBatch(graphs)
        br = BatchRunner(b)
        br.enqueue()
        assert br.results()[0] == want
    # an empty batch
    b = PackedBatch([])
    br = BatchRunner(b)
    br.enqueue()
    assert br.results() == ([], 0)
    # vertices outside every graph range add to no graph total
    g = [tuple(torch.tensor(x, dtype=torch.int32) for x in pins.complete(4)[1:]) + (4,),
         tuple(torch.tensor(x, dtype=torch.int32) for x in pins.complete(5)[1:]) + (5,)]
    b = PackedBatch(g)
    br = BatchRunner(b)
    torch.cuda.synchronize()
    b.vtx_off = torch.tensor([0, 4], dtype=torch.int64, device="cuda")  # graph 1 left out
    b.G = 1
    br.enqueue()
    totals, grand = br.results()
    assert totals == [4] and grand == 4 + 10
    with pytest.raises(_lib.TcError):
        _lib.tc_count_batched(b.n, br.dag_ptr, br.dag_col, b.vtx_off, br.totals[:1], br.ws_count,
                              tune={"small_max": 97})


def _t_digest(t: np.ndarray) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(t, dtype="<u8").tobytes()).hexdigest()[:16]


@pytest.mark.slow
def test_full_batch_4096_against_oracle(tc):
    """The whole 4096-graph batch (n log-uniform in [2^8, 2^16], average degree U(4, 64), half
    Erdos-Renyi and half R-MAT; sum n = 4.7e7 > 2^24, so the folded wide hash runs; int32
    offsets, as 2 * pairs < 2^31) as the benchmark runs it, a HIP-graph replay: every graph's
    total and every t(v) of every graph against the oracle's stored counts
    (tests/golden/make_batch4096.py: totals and a digest of each graph's t), the tuned
    total-only launch too, and a stratified
    sample of graphs (the largest by edges and by vertices, and random ones) recounted here by
    the oracle, totals and t(v); then every total again with int64 offsets."""
    import json
    import os
    import time

    from paper_1909_02127_amd.batch import BatchRunner, PackedBatch
    from tests import goldens
    with open(os.path.join(goldens.GOLDEN_DIR, "batch4096_seed4.json")) as f:
        gold = json.load(f)["graphs"]
    specs = graphgen.batch_suite_spec(4096, seed=4)
    t0 = time.perf_counter()
    graphs = []
    for i, g in enumerate(specs):
        graphs.append(graphgen.batch_graph(g, device="cuda"))
        if (i + 1) % 1024 == 0:
            _say(f"batch 4096: generated {i + 1} graphs ({time.perf_counter() - t0:.0f}s)")
    b = PackedBatch(graphs)  # the benchmark's choice: int32 offsets (2 * pairs < 2^31)
    assert b.offset_bytes == 4
    assert b.n > (1 << 24)
    assert b.graph_edges() == [g["m"] for g in gold]
    want = [g["triangles"] for g in gold]
    br = BatchRunner(b, per_vertex=True)
    br.capture()
    br.totals.fill_(-1)
    br.replay()
    totals, grand = br.results()
    assert totals == want
    assert grand == sum(want)
    pv = br.pv[: b.n].cpu().numpy().view(np.uint64)
    off = b.vtx_off.cpu().numpy()
    bad = [i for i, g in enumerate(gold) if _t_digest(pv[off[i]: off[i + 1]]) != g["t_digest"]]
    assert not bad, f"t digests differ for graphs {bad[:10]}"
    _say(f"batch 4096: totals and t of all graphs match ({time.perf_counter() - t0:.0f}s)")
    # total-only launches: default and the split the tuner picks on this batch
    for tune in (None, {"small_max": 96}):
        bt = BatchRunner(b, tune=tune)
        bt.capture()
        bt.replay()
        assert bt.results()[0] == want, tune
        del bt
    # live oracle on a stratified sample
    ms = np.array([g["m"] for g in gold])
    ns = np.array([g["n"] for g in gold])
    rng = np.random.default_rng(4)
    pick = sorted(set(np.argsort(-ms)[:3].tolist()) | set(np.argsort(-ns)[:2].tolist())
                  | set(rng.choice(len(gold), 6, replace=False).tolist()))
    for i in pick:
        s, d, n = graphs[i]
        T, t = oracle.triangles(n, s.cpu().numpy(), d.cpu().numpy(), per_vertex=True)
        assert T == totals[i], i
        np.testing.assert_array_equal(pv[off[i]: off[i + 1]], t)
    _say(f"batch 4096: live oracle on {len(pick)} graphs ({time.perf_counter() - t0:.0f}s)")
    # the same union with int64 offsets: every total again
    del br, pv
    b8 = PackedBatch(graphs, offset_bytes=8)
    del b
    br8 = BatchRunner(b8)
    br8.capture()
    br8.replay()
    assert br8.results()[0] == want
    _say(f"batch 4096: int64 offsets match ({time.perf_counter() - t0:.0f}s)")
