"""CPU emulation of how the 4-clique kernel (clique4.hip, tc_count_k4) splits heavy sources.

A pre-pass gives each source u with d+(u) >= 3 its wedge work w(u), the sum of d+(v) over its
middles with d+(v) >= 2, and, when w(u) > 8192, ceil(w / 8192) parts (at most 64, and at most
one per group of four middles).  Each source gets a contiguous range of a task array of
n / 2 + 4096 entries (a wave reserves the ranges of up to 64 such sources with one atomic add,
in lane order, which is one of the orders emulated here); if the range fits the source writes one
task (u, part, parts) per entry and is marked as split, otherwise it blanks the entries of its
range that lie below the capacity and stays whole.  Workgroups take the first min(reserved, capacity) entries, skipping
blanks, then every unmarked source whole; part k of P takes the middles iv whose group iv // 4
is k mod P (four waves, one middle each per group).

The emulation runs the reservations in random orders (the atomics' order on the device is not
fixed), with the capacity shrunk so that some reservations do not fit, and checks that every
middle of every source is taken exactly once, that no entry below the cut is left unwritten and
that the part counts follow the rule.
"""
import numpy as np
import pytest

PART_WORK = 8192
MAX_PARTS = 64
WAVES = 4


def parts_of(du, w):
    if du < 3:
        return 0
    p = -(-w // PART_WORK)
    p = min(p, MAX_PARTS, -(-du // WAVES))
    return p if p > 1 else 0


def emulate(dplus, rp, col, cap, order):
    n = dplus.size
    w = np.array([sum(int(dplus[v]) for v in col[rp[u]:rp[u + 1]] if dplus[v] >= 2)
                  for u in range(n)], dtype=np.int64)
    parts = np.array([parts_of(int(dplus[u]), int(w[u])) for u in range(n)])
    tasks = [None] * cap
    split = np.zeros(n, dtype=bool)
    counter = 0
    for u in order:
        p = int(parts[u])
        if p == 0:
            continue
        at, counter = counter, counter + p
        if at + p <= cap:
            for k in range(p):
                tasks[at + k] = (u, k, p)
            split[u] = True
        else:
            for k in range(p):
                if at + k < cap:
                    tasks[at + k] = (-1, 0, 0)
    taken = {}
    for t in range(min(counter, cap)):
        assert tasks[t] is not None, "an entry below the cut was never written"
        u, k, p = tasks[t]
        if u < 0:
            continue
        for iv in range(int(dplus[u])):
            if (iv // WAVES) % p == k:
                taken[(u, iv)] = taken.get((u, iv), 0) + 1
    for u in range(n):
        if split[u] or dplus[u] < 3:
            continue
        for iv in range(int(dplus[u])):
            taken[(u, iv)] = taken.get((u, iv), 0) + 1
    return parts, split, taken, counter


def random_lists(rng, n):
    """Random out-lists (any vertex but u; the split rule does not need a DAG) with a few
    heavy sources: many middles of high out-degree."""
    dplus = rng.choice([0, 1, 2, 5, 30, 200, 1500], size=n, p=[.2, .2, .2, .2, .1, .07, .03])
    rows = [np.sort(rng.choice(np.delete(np.arange(n), u), size=int(dplus[u]), replace=False))
            for u in range(n)]
    rp = np.concatenate([[0], np.cumsum(dplus)])
    return dplus, rp, np.concatenate(rows)


@pytest.mark.parametrize("seed", range(4))
def test_k4_split_covers_every_middle_once(seed):
    rng = np.random.default_rng(seed)
    n = 2500
    dplus, rp, col = random_lists(rng, n)
    for cap_name in ("fits", "overflows"):
        order = rng.permutation(n)
        full = n // 2 + 4096
        parts_all = None
        for cap in ((full,) if cap_name == "fits" else (5, 97, 300)):
            parts, split, taken, reserved = emulate(dplus, rp, col, cap, order)
            parts_all = parts
            want = {(u, iv) for u in range(n) if dplus[u] >= 3 for iv in range(int(dplus[u]))}
            assert set(taken) == want
            assert all(c == 1 for c in taken.values())
            if cap_name == "fits":
                assert reserved <= cap and split.sum() == (parts > 0).sum()
            else:
                # some reservations do not fit (with 5 entries, none does)
                assert reserved > cap and split.sum() < (parts > 0).sum()
                assert (split.sum() > 0) == (cap > 5)
        assert (parts_all > 0).sum() >= 10  # the graph has split sources at all
        assert parts_all.max() <= MAX_PARTS


def test_k4_part_rule():
    assert parts_of(2, 10 ** 9) == 0          # not a 4-clique source
    assert parts_of(100, PART_WORK) == 0      # at the threshold: whole
    assert parts_of(100, PART_WORK + 1) == 2
    assert parts_of(8, 10 ** 9) == 2          # at most one part per four middles
    assert parts_of(10 ** 4, 10 ** 9) == MAX_PARTS
