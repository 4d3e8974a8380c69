"""Host emulation of the index arithmetic of the concatenated short-list walk (count kernel:
two 64-lane windows per step; 4-clique kernel: one), checked on the CPU.

Each lane holds one list (row start vb, length len >= 0).  The lists are laid end to end by an
exclusive scan of the lengths; every non-empty list marks its first walk position, an inclusive
max-scan of the marks (carried from window to window) gives each position its list sk, and the
position reads col[pos + (vb[sk] - start[sk])].  The kernels rely on this landing inside list sk
for every pos < total without a per-lane length check; this test checks that claim exhaustively
over random and degenerate length vectors."""
import numpy as np
import pytest

WAVE = 64


def walk_indices(lens, vb, win):
    lens = np.asarray(lens, dtype=np.int64)
    incl = np.cumsum(lens)
    start = incl - lens
    total = int(incl[-1])
    delta = vb - start
    mark = np.full(win * WAVE, -1, dtype=np.int64)
    carry = -1
    out = []
    for base in range(0, total, win * WAVE):
        marks = (lens > 0) & (start >= base) & (start < base + win * WAVE)
        lanes = np.nonzero(marks)[0]
        mark[start[lanes] - base] = lanes
        for k in range(win):
            sk = np.maximum.accumulate(mark[k * WAVE:(k + 1) * WAVE])
            sk = np.maximum(sk, carry)
            carry = int(sk[-1])
            pos = base + k * WAVE + np.arange(WAVE)
            src = np.where(sk < 0, 0, sk)
            at = pos + delta[src]
            ok = pos < total
            out.append((pos[ok], src[ok], at[ok]))
        mark[start[lanes] - base] = -1
    assert (mark == -1).all()  # markers are left cleared for the next walk
    return total, out


def check(lens, win, rng):
    lens = np.asarray(lens, dtype=np.int64)
    vb = rng.integers(0, 1 << 30, size=WAVE).astype(np.int64)
    total, parts = walk_indices(lens, vb, win)
    seen = 0
    incl = np.cumsum(lens)
    start = incl - lens
    for pos, src, at in parts:
        # the position's list is the one whose range [start, start + len) holds it
        assert (lens[src] > 0).all()
        assert (start[src] <= pos).all() and (pos < start[src] + lens[src]).all()
        assert (vb[src] <= at).all() and (at < vb[src] + lens[src]).all()
        seen += pos.size
    assert seen == total


@pytest.mark.parametrize("win", [1, 2])
def test_random_length_vectors(win):
    rng = np.random.default_rng(7 + win)
    for _ in range(400):
        zero_frac = rng.choice([0.0, 0.3, 0.9])
        lens = rng.integers(1, 64, size=WAVE)
        lens[rng.random(WAVE) < zero_frac] = 0
        if lens.sum() == 0:
            lens[rng.integers(WAVE)] = 1
        check(lens, win, rng)


@pytest.mark.parametrize("win", [1, 2])
def test_degenerate_length_vectors(win):
    rng = np.random.default_rng(3)
    one_last = np.zeros(WAVE, dtype=np.int64)
    one_last[-1] = 1
    one_first = np.zeros(WAVE, dtype=np.int64)
    one_first[0] = 63
    leading_zeros = np.concatenate([np.zeros(40, dtype=np.int64), np.full(24, 63)])
    cases = [np.ones(WAVE, dtype=np.int64), np.full(WAVE, 63), one_last, one_first, leading_zeros,
             np.tile([0, 64], WAVE // 2), np.full(WAVE, 2)]
    for lens in cases:
        check(lens, win, rng)
