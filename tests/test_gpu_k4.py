"""GPU parity of tc_count_k4 (the 4-clique query) against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests import goldens, pins

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


def _dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.int32)).cuda()


def _gpu_k4(tc, n, s, d, order=0, offset_bytes=4):
    from paper_1909_02127_amd import _lib
    p = tc.Pipeline(n, max(len(s), 1), offset_bytes=offset_bytes, order=order)
    p.build(_dev(s), _dev(d))
    p.orient()
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(_lib.tc_count_k4_workspace(n), dtype=torch.uint8, device="cuda")
    _lib.tc_count_k4(n, p.dag_ptr, p.dag_col, total, ws)
    torch.cuda.synchronize()
    return int(total.item())


def _check(tc, n, s, d, order=0, offset_bytes=4):
    assert _gpu_k4(tc, n, s, d, order, offset_bytes) == oracle.k4(n, np.asarray(s), np.asarray(d),
                                                                  order=order)


@pytest.mark.parametrize("fx", goldens.all_fixtures(), ids=lambda f: f.name)
def test_k4_golden_fixtures(tc, fx):
    for order in (0, 1):
        _check(tc, fx.n, fx.src, fx.dst, order, 4 + 4 * order)


def test_k4_closed_forms(tc):
    from math import comb
    for n in (4, 7, 30, 90):
        _, s, d = pins.complete(n)
        for order in (0, 1):
            assert _gpu_k4(tc, n, s, d, order) == comb(n, 4)
    for r in (3, 6):
        n, s, d = pins.wheel(r)
        assert _gpu_k4(tc, n, s, d) == (1 if r == 3 else 0)


def test_k4_random_tiny(tc):
    for seed in range(30):
        rng = np.random.default_rng(2100 + seed)
        n = int(rng.integers(1, 40))
        n, s, d = pins.random_simple(n, float(rng.choice([0.2, 0.5, 0.8])), seed)
        n, s, d = pins.noisy(n, s, d, seed)
        _say("k4 tiny seed", seed, "n", n)
        for order in (0, 1):
            _check(tc, n, s, d, order, 4 + 4 * (seed % 2))


@pytest.mark.parametrize("scale,seed", [(10, 1), (13, 2), (15, 3)])
def test_k4_rmat(tc, scale, seed):
    s, d, n = graphgen.rmat(scale, 16, seed)
    _say("k4 rmat", scale)
    for order in (0, 1):
        _check(tc, n, s.numpy(), d.numpy(), order)


def test_k4_long_out_lists(tc):
    """Id order gives vertex 0 an out-list beyond the LDS copy (the in-memory path), with
    enough common neighbours to fill the kept-w list more than once."""
    rng = np.random.default_rng(5)
    n = 3001
    dense = np.arange(1, 1501)
    s = np.concatenate([np.zeros(n - 1, dtype=np.int64), np.ones(1999, dtype=np.int64),
                        rng.integers(1, n, 20000), np.repeat(dense[:60], 60)])
    d = np.concatenate([np.arange(1, n), np.arange(2, 2001), rng.integers(1, n, 20000),
                        np.tile(dense[:60], 60)])
    for order in (0, 1):
        _check(tc, n, s, d, order)


def test_k4_split_sources(tc):
    """The kernel splits a source whose wedge work (the sum of d+(v) over its middles with
    d+(v) >= 2) passes 8192 over several workgroups, as tasks of one part of its middles
    each, in an array of n / 2 + 4096 entries; sources whose tasks do not fit stay whole.
    K_800 and K_1000 in degree order split several hundred sources into more tasks than
    that array holds (10674 against 4496 for K_800), so split and whole heavy sources share
    a launch, with N+(u) hashed (d+ <= 816) or sorted (K_1000's first sources).  R-MAT
    scale 15 in id order splits 1805 sources into 6642 tasks, all of which fit."""
    from math import comb
    for n in (800, 1000):
        _, s, d = pins.complete(n)
        _say("k4 split K", n)
        for order, ob in ((0, 4), (1, 8)):
            assert _gpu_k4(tc, n, s, d, order, ob) == comb(n, 4), (n, order)
    s, d, n = graphgen.rmat(15, 16, 3)
    _say("k4 split rmat 15")
    _check(tc, n, s.numpy(), d.numpy(), 1, 8)


def test_k4_empty_and_small(tc):
    for n, s, d in [(0, [], []), (1, [], []), (3, [0, 1, 2], [1, 2, 0]), (4, [0, 0, 0, 1, 1, 2],
                                                                         [1, 2, 3, 2, 3, 3])]:
        _check(tc, n, s, d)


def _colliding_ids(count: int, bits: int = 4) -> list[int]:
    """`count` ids below 2^24 whose 24-bit product with the table multiplier agrees in
    its top 2 * bits bits: in a table with 2^bits slots per half they all share one
    slot pair, so a cuckoo insertion of three of them cannot succeed."""
    buckets: dict[int, list[int]] = {}
    for x in range(1 << 20, 1 << 24):
        key = ((x * 0x9E3779) & 0xFFFFFFFF) >> (32 - 2 * bits)
        buckets.setdefault(key, []).append(x)
        if len(buckets[key]) == count:
            return buckets[key]
    raise AssertionError("no colliding ids found")


def test_k4_hash_insertion_failure_falls_back(tc):
    """A source whose out-neighbours all share one slot pair overflows the cuckoo table;
    the kernel must fall back to the sorted copy and still count exactly."""
    xs = _colliding_ids(3)
    _say("colliding ids", xs)
    # K4 on {0} + xs (vertex 0 is the lowest rank: all degrees equal, ties by id), plus a
    # K5 elsewhere so the graph also has ordinary sources
    verts = [0] + xs
    s = [a for i, a in enumerate(verts) for b in verts[i + 1:]]
    d = [b for i, a in enumerate(verts) for b in verts[i + 1:]]
    k5 = list(range(10, 15))
    s += [a for i, a in enumerate(k5) for b in k5[i + 1:]]
    d += [b for i, a in enumerate(k5) for b in k5[i + 1:]]
    n = max(xs) + 1
    got = _gpu_k4(tc, n, s, d)
    assert got == oracle.k4(n, np.asarray(s), np.asarray(d)) == 1 + 5
