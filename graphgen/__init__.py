"""Seeded synthetic graph inputs: Erdos-Renyi G(n, m), R-MAT, the packed batch suite
and Poisson request arrivals.

This module only draws endpoint pairs.  It holds none of the triangle-counting
arithmetic (no cleaning of the pairs it hands out for single-graph workloads, no
orientation, no counting), so both the CPU oracle and the GPU path can consume
its output without sharing any part of the method.

Randomness is counter based: every draw is ``mix(seed, stream, index)`` where
``mix`` is the MurmurHash3 32-bit finaliser (Appleby, "fmix32") applied twice.
On the CPU it runs as numpy uint32 arithmetic (wrapping multiply); on a device
as torch int64 element-wise ops whose intermediate values stay below 2**63.
Both compute the same function, so a call gives bit-identical pairs on the CPU
and on a GPU, and large workloads can be generated directly in device memory.

The paper evaluates on HPEC Graph Challenge graphs (real-world SNAP graphs and
graph500 R-MAT graphs, scale 18-21, edge factor 16; experiments section and
Table 1).  Those files are not used here: R-MAT with the graph500 parameters
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05) and Erdos-Renyi graphs stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

__all__ = [
    "mix_u32",
    "uniform_u32",
    "erdos_renyi",
    "rmat",
    "rmat_unique",
    "random_permutation",
    "batch_suite_spec",
    "batch_graph",
    "poisson_arrivals",
    "GraphSpec",
]

_M32 = 0xFFFFFFFF
_FMIX_C1 = 0x85EBCA6B
_FMIX_C2 = 0xC2B2AE35
_GOLDEN = 0x9E3779B1


def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    """(x * c) mod 2**32 for 0 <= x < 2**32, split so no int64 product overflows."""
    lo = x * (c & 0xFFFF)
    hi = ((x * (c >> 16)) & 0xFFFF) << 16
    return (lo + hi) & _M32


def _fmix32(x: torch.Tensor) -> torch.Tensor:
    x = x ^ (x >> 16)
    x = _mul32(x, _FMIX_C1)
    x = x ^ (x >> 13)
    x = _mul32(x, _FMIX_C2)
    x = x ^ (x >> 16)
    return x


def _fmix32_int(x: int) -> int:
    x &= _M32
    x ^= x >> 16
    x = (x * _FMIX_C1) & _M32
    x ^= x >> 13
    x = (x * _FMIX_C2) & _M32
    x ^= x >> 16
    return x


def _stream_key(seed: int, stream: int) -> tuple[int, int]:
    k1 = _fmix32_int((seed * _GOLDEN + 0x632BE5AB) ^ _fmix32_int(stream + 0x1B873593))
    k2 = _fmix32_int(k1 + 0x7F4A7C15 + (seed >> 32))
    return k1, k2


def _fmix32_np(x: np.ndarray) -> np.ndarray:
    """In-place fmix32 on a uint32 array (numpy unsigned multiply wraps mod 2**32)."""
    x ^= x >> np.uint32(16)
    x *= np.uint32(_FMIX_C1)
    x ^= x >> np.uint32(13)
    x *= np.uint32(_FMIX_C2)
    x ^= x >> np.uint32(16)
    return x


def mix_u32(idx: torch.Tensor, seed: int, stream: int) -> torch.Tensor:
    """32-bit pseudo-random word (as int64) for each counter in ``idx`` (int64, < 2**32).

    CPU tensors go through numpy uint32 arithmetic, device tensors through the
    overflow-free int64 split multiply; both compute the same function.
    """
    k1, k2 = _stream_key(seed, stream)
    if idx.device.type == "cpu":
        x = idx.numpy().astype(np.uint32) ^ np.uint32(k1)
        _fmix32_np(x)
        x ^= np.uint32(k2)
        _fmix32_np(x)
        return torch.from_numpy(x.astype(np.int64))
    x = _fmix32((idx & _M32) ^ k1)
    x = _fmix32(x ^ k2)
    return x


def mix_u32_device_path(idx: torch.Tensor, seed: int, stream: int) -> torch.Tensor:
    """The int64 split-multiply path on any device (used to check both paths agree)."""
    k1, k2 = _stream_key(seed, stream)
    return _fmix32(_fmix32((idx & _M32) ^ k1) ^ k2)


def uniform_u32(num: int, seed: int, stream: int, *, start: int = 0, device="cpu") -> torch.Tensor:
    idx = torch.arange(start, start + num, dtype=torch.int64, device=device)
    return mix_u32(idx, seed, stream)


def vertex_labels(n: int, k: int, seed: int, *, device="cpu") -> torch.Tensor:
    """A label in [0, k) for each of n vertices (int32), uniform, from counter-based words."""
    if k < 1:
        raise ValueError("k >= 1 labels")
    return (uniform_u32(n, seed, stream=0x1AB, device=device) % k).to(torch.int32)


def random_permutation(n: int, seed: int, *, device="cpu") -> torch.Tensor:
    """A seeded permutation of [0, n): argsort of counter-based keys (ties by index)."""
    keys = uniform_u32(n, seed, stream=0x5EED) * n + torch.arange(n, dtype=torch.int64)
    keys = keys.to(device)
    return torch.argsort(keys, stable=True)


def _rmat_block(num: int, scale: int, seed: int, start: int, a: float, b: float, c: float,
                device) -> tuple[torch.Tensor, torch.Tensor]:
    ta = int(math.floor(a * 2**32))
    tab = int(math.floor((a + b) * 2**32))
    tabc = int(math.floor((a + b + c) * 2**32))
    idx = torch.arange(start, start + num, dtype=torch.int64, device=device)
    src = torch.zeros(num, dtype=torch.int64, device=device)
    dst = torch.zeros(num, dtype=torch.int64, device=device)
    for level in range(scale):
        x = mix_u32(idx, seed, stream=1000 + level)
        bit = 1 << (scale - 1 - level)
        # quadrants: [0,a) -> (0,0); [a,a+b) -> (0,1); [a+b,a+b+c) -> (1,0); rest -> (1,1)
        row_bit = x >= tab
        col_bit = ((x >= ta) & (x < tab)) | (x >= tabc)
        src += row_bit.to(torch.int64) * bit
        dst += col_bit.to(torch.int64) * bit
        del x, row_bit, col_bit
    return src, dst


def rmat(scale: int, edge_factor: int = 16, seed: int = 0, *, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, permute: bool = True, device="cpu") -> tuple[torch.Tensor, torch.Tensor, int]:
    """Raw R-MAT pairs: edge_factor * 2**scale samples, no noise, seeded vertex permutation.

    The pairs are returned as drawn: they include self-loops, duplicates and both
    directions of some edges.  Cleaning them is the job of the consumer.
    Returns (src, dst, n) with int32 tensors on ``device`` and n = 2**scale.
    """
    n = 1 << scale
    num = edge_factor * n
    src, dst = _rmat_block(num, scale, seed, 0, a, b, c, device)
    if permute:
        perm = random_permutation(n, seed ^ 0xA5A5, device=device)
        src = perm[src]
        dst = perm[dst]
    return src.to(torch.int32), dst.to(torch.int32), n


def _first_unique(keys: torch.Tensor, limit: int) -> torch.Tensor:
    """Positions of the first occurrence of each distinct key, in draw order, at most ``limit``."""
    order = torch.argsort(keys, stable=True)
    sk = keys[order]
    first = torch.ones_like(sk, dtype=torch.bool)
    if sk.numel() > 1:
        first[1:] = sk[1:] != sk[:-1]
    pos = torch.sort(order[first]).values
    return pos[:limit]


def erdos_renyi(n: int, m: int, seed: int = 0, *, device="cpu") -> tuple[torch.Tensor, torch.Tensor, int]:
    """G(n, m): uniform over simple graphs with exactly m edges (m <= n(n-1)/2).

    Candidate pairs are drawn i.i.d. uniform, self-loops rejected, and the first m
    distinct unordered pairs in draw order are kept (seeded rejection sampling).
    Returns (src, dst, n) int32, one entry per undirected edge, endpoints in draw order.
    """
    if n < 0 or m < 0 or m > n * (n - 1) // 2:
        raise ValueError(f"G(n={n}, m={m}) is impossible")
    if m == 0:
        z = torch.zeros(0, dtype=torch.int32, device=device)
        return z, z.clone(), n
    drawn = 0
    a_all, b_all = [], []
    have = 0
    while True:
        chunk = max(64, int(1.25 * (m - have)) + 64)
        ua = uniform_u32(chunk, seed, 1, start=drawn, device=device)
        ub = uniform_u32(chunk, seed, 2, start=drawn, device=device)
        drawn += chunk
        a = (ua * n) >> 32
        b = (ub * n) >> 32
        ok = a != b
        a_all.append(a[ok])
        b_all.append(b[ok])
        A = torch.cat(a_all)
        B = torch.cat(b_all)
        keys = torch.minimum(A, B) * n + torch.maximum(A, B)
        pos = _first_unique(keys, m)
        have = pos.numel()
        if have >= m:
            return A[pos].to(torch.int32), B[pos].to(torch.int32), n
        if drawn > 64 * m + 4096:
            raise RuntimeError("G(n, m) rejection sampling did not converge")


def rmat_unique(n: int, m_target: int, seed: int = 0, *, a: float = 0.57, b: float = 0.19,
                c: float = 0.19, max_rounds: int = 64, device="cpu") -> tuple[torch.Tensor, torch.Tensor, int]:
    """R-MAT graph on n vertices (n need not be a power of two) with ~m_target unique edges.

    scale = ceil(log2 n); samples with an endpoint >= n and self-loops are rejected,
    and distinct unordered pairs are kept in draw order until m_target is reached
    (capped at n(n-1)/2).  Heavy skew can starve the last distinct pairs: after
    ``max_rounds`` oversampling rounds the graph keeps what it has.  The vertex
    ids are then permuted.  Returns one entry per undirected edge.
    """
    m_target = min(m_target, n * (n - 1) // 2)
    scale = max(1, math.ceil(math.log2(max(n, 2))))
    drawn = 0
    S, D = [], []
    pos = torch.zeros(0, dtype=torch.int64, device=device)
    A = B = torch.zeros(0, dtype=torch.int64, device=device)
    for _ in range(max_rounds):
        need = m_target - pos.numel()
        if need <= 0:
            break
        chunk = max(1024, 2 * need)
        s, d = _rmat_block(chunk, scale, seed, drawn, a, b, c, device)
        drawn += chunk
        ok = (s < n) & (d < n) & (s != d)
        S.append(s[ok])
        D.append(d[ok])
        A = torch.cat(S)
        B = torch.cat(D)
        keys = torch.minimum(A, B) * n + torch.maximum(A, B)
        pos = _first_unique(keys, m_target)
    perm = random_permutation(n, seed ^ 0xA5A5, device=device)
    return perm[A[pos]].to(torch.int32), perm[B[pos]].to(torch.int32), n


@dataclass(frozen=True)
class GraphSpec:
    index: int
    kind: str  # "er" or "rmat"
    n: int
    avg_degree: float
    m_target: int
    seed: int


def batch_suite_spec(count: int = 4096, seed: int = 4, *, log2_min: int = 8, log2_max: int = 16,
                     deg_min: float = 4.0, deg_max: float = 64.0) -> list[GraphSpec]:
    """The packed-batch workload: n log-uniform in [2**log2_min, 2**log2_max], average
    degree uniform in [deg_min, deg_max], Erdos-Renyi for even i and R-MAT for odd i."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.Generator(np.random.PCG64(ss))
        n = int(math.floor(math.exp(rng.uniform(math.log(2**log2_min), math.log(2**log2_max)))))
        n = max(2, n)
        d = float(rng.uniform(deg_min, deg_max))
        m = min(int(round(n * d / 2)), n * (n - 1) // 2)
        g_seed = int(ss.generate_state(1, dtype=np.uint64)[0] & 0xFFFFFFFFFFFF)
        out.append(GraphSpec(i, "er" if i % 2 == 0 else "rmat", n, d, m, g_seed))
    return out


def batch_graph(spec: GraphSpec, *, device="cpu") -> tuple[torch.Tensor, torch.Tensor, int]:
    if spec.kind == "er":
        return erdos_renyi(spec.n, spec.m_target, spec.seed, device=device)
    return rmat_unique(spec.n, spec.m_target, spec.seed, device=device)


def poisson_arrivals(count: int, qps: float, seed: int = 5) -> np.ndarray:
    """Open-loop arrival times (seconds from 0) with exponential gaps at rate ``qps``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=count))
