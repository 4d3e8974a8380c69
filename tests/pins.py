"""Independent checks used to pin the oracle (test helpers; no oracle code here).

Each helper computes triangle counts from first principles by a route that
shares nothing with the oracle's node iterator:
  - brute force over all vertex triples (Def. 2 with Q = K3),
  - trace(A^3)/6 and diag(A^3)/2 with exact integer matrix products,
  - closed forms for graph families.
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np


def edge_set(src, dst) -> set[frozenset]:
    return {frozenset((int(a), int(b))) for a, b in zip(src, dst) if int(a) != int(b)}


def brute_force(n: int, src, dst) -> tuple[int, np.ndarray]:
    """Every unordered triple {i, j, k} whose three pairs are edges is a triangle."""
    adj = [set() for _ in range(n)]
    for e in edge_set(src, dst):
        a, b = tuple(e)
        adj[a].add(b)
        adj[b].add(a)
    t = np.zeros(n, dtype=np.uint64)
    total = 0
    for i, j, k in itertools.combinations(range(n), 3):
        if j in adj[i] and k in adj[i] and k in adj[j]:
            total += 1
            t[i] += 1
            t[j] += 1
            t[k] += 1
    return total, t


def brute_force_sets(n: int, src, dst) -> list[tuple[int, int, int]]:
    """Every triangle {a, b, c} as a sorted triple, by checking all vertex triples."""
    e = edge_set(src, dst)
    out = []
    for a in range(n):
        for b in range(a + 1, n):
            if frozenset((a, b)) not in e:
                continue
            for c in range(b + 1, n):
                if frozenset((a, c)) in e and frozenset((b, c)) in e:
                    out.append((a, b, c))
    return out


def brute_force_k4(n: int, src, dst) -> int:
    """4-cliques by checking every 4-subset of the vertices."""
    import itertools
    e = edge_set(src, dst)
    nb = [set() for _ in range(n)]
    for a, b in (tuple(x) for x in e):
        nb[a].add(b)
        nb[b].add(a)
    count = 0
    for a, b in (tuple(sorted(x)) for x in e):
        common = sorted(w for w in nb[a] & nb[b] if w > b)
        for c, d in itertools.combinations(common, 2):
            if d in nb[c]:
                count += 1
    return count


def trace_cube(n: int, src, dst) -> tuple[int, np.ndarray]:
    """T = trace(A^3)/6 and t = diag(A^3)/2 for the 0/1 symmetric adjacency A."""
    A = np.zeros((n, n), dtype=np.float64)
    for e in edge_set(src, dst):
        a, b = tuple(e)
        A[a, b] = A[b, a] = 1.0
    # float64 products of 0/1 matrices are exact while entries stay below 2**53
    # (here at most n**2); the exactness is asserted before converting.
    A2 = A @ A
    diag_f = np.einsum("ij,ji->i", A2, A)
    assert n < 2**20 and np.all(diag_f == np.round(diag_f))
    diag = diag_f.astype(np.int64)
    tr = int(diag.sum())
    assert tr % 6 == 0 and np.all(diag % 2 == 0)
    return tr // 6, (diag // 2).astype(np.uint64)


# ---- graph families with closed-form counts ---------------------------------

def complete(n):
    e = list(itertools.combinations(range(n), 2))
    return n, [a for a, _ in e], [b for _, b in e]


def cycle(n):
    return n, list(range(n)), [(i + 1) % n for i in range(n)]


def wheel(rim):
    """Hub 0 plus a rim cycle on 1..rim."""
    s = [0] * rim + [1 + i for i in range(rim)]
    d = [1 + i for i in range(rim)] + [1 + (i + 1) % rim for i in range(rim)]
    return rim + 1, s, d


def star(leaves):
    return leaves + 1, [0] * leaves, list(range(1, leaves + 1))


def complete_bipartite(a, b):
    s, d = [], []
    for i in range(a):
        for j in range(b):
            s.append(i)
            d.append(a + j)
    return a + b, s, d


def complete_tripartite(a, b, c):
    parts = [list(range(0, a)), list(range(a, a + b)), list(range(a + b, a + b + c))]
    s, d = [], []
    for p, q in itertools.combinations(range(3), 2):
        for i in parts[p]:
            for j in parts[q]:
                s.append(i)
                d.append(j)
    return a + b + c, s, d


def friendship(k):
    """k triangles sharing the centre 0."""
    s, d = [], []
    for i in range(k):
        x, y = 1 + 2 * i, 2 + 2 * i
        s += [0, 0, x]
        d += [x, y, y]
    return 2 * k + 1, s, d


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    e = outer + spokes + inner
    return 10, [a for a, _ in e], [b for _, b in e]


def closed_form_cases():
    """(name, (n, src, dst), T, t or None)"""
    cases = []
    for n in range(0, 13):
        t = np.full(n, comb(n - 1, 2) if n >= 1 else 0, dtype=np.uint64)
        cases.append((f"K{n}", complete(n), comb(n, 3), t))
    for n in range(3, 12):
        cases.append((f"C{n}", cycle(n), 1 if n == 3 else 0, None))
    for r in range(3, 12):
        T = 4 if r == 3 else r
        t = None if r == 3 else np.array([r] + [2] * r, dtype=np.uint64)
        cases.append((f"W{r}", wheel(r), T, t))
    for k in range(0, 9):
        cases.append((f"star{k}", star(k), 0, None))
    for a, b in [(1, 1), (2, 3), (3, 3), (4, 7)]:
        cases.append((f"K{a},{b}", complete_bipartite(a, b), 0, None))
    for a, b, c in [(1, 1, 1), (2, 2, 2), (1, 2, 3), (3, 4, 5)]:
        cases.append((f"K{a},{b},{c}", complete_tripartite(a, b, c), a * b * c, None))
    for k in range(0, 7):
        t = np.array([k] + [1] * (2 * k), dtype=np.uint64)
        cases.append((f"F{k}", friendship(k), k, t))
    cases.append(("petersen", petersen(), 0, None))
    cases.append(("empty-n5", (5, [], []), 0, np.zeros(5, dtype=np.uint64)))
    cases.append(("n1", (1, [], []), 0, np.zeros(1, dtype=np.uint64)))
    return cases


def random_simple(n: int, p: float, seed: int):
    rng = np.random.default_rng(seed)
    s, d = [], []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < p:
                if rng.random() < 0.5:
                    s.append(i)
                    d.append(j)
                else:
                    s.append(j)
                    d.append(i)
    return n, s, d


def noisy(n, src, dst, seed):
    """Same edge set with duplicates, reversed copies and self-loops added, shuffled."""
    rng = np.random.default_rng(seed)
    s, d = list(src), list(dst)
    for a, b in zip(list(src), list(dst)):
        r = rng.random()
        if r < 0.3:
            s.append(b)
            d.append(a)
        elif r < 0.5:
            s.append(a)
            d.append(b)
    for _ in range(max(1, n // 3)):
        if n:
            v = int(rng.integers(n))
            s.append(v)
            d.append(v)
    perm = rng.permutation(len(s))
    return n, [s[i] for i in perm], [d[i] for i in perm]
