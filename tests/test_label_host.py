"""CPU emulation of the label filter's indexing (label.hip, tc_count_labelled).

One wave takes 32 consecutive rows and walks their edges as one contiguous column range, 64
edges per step.  A lane finds its edge's row from LDS marks: every non-empty row writes
(row << 6 | position) at its first position in the step, a max-scan over the lanes gives each
lane the last row starting at or before it and where that row's part of the step begins, and
the last lane of the previous step carries its row (from position 0) into the next.  The last
lane of each row's part adds the part's kept edges (a ballot masked to the part) to the row's
counter; the compaction places each kept edge at its row's new offset plus the row's kept
edges of earlier steps plus those of lower lanes in its part.

The emulation runs those rules lane by lane on random CSR rows (empty rows, rows spanning
several steps, rows shorter than a step) and checks the kept degrees and the compacted columns
against a row-by-row filter written from the definition, and that every output slot is written
exactly once and inside the kept total.
"""
import numpy as np
import pytest

W, ROWS, STEPS = 64, 32, 4


def popc(x):
    return bin(x).count("1")


def lane_range(lo, hi):
    up_hi = (1 << 64) - 1 if hi >= W else (1 << hi) - 1
    up_lo = (1 << lo) - 1
    return up_hi & ~up_lo & ((1 << 64) - 1) if hi > lo else 0


def fits(q, x, y):
    lo, hi = min(x, y), max(x, y)
    return (lo == q[0] and (hi == q[1] or hi == q[2])) or (lo == q[1] and hi == q[2])


def walk_rows(bnd, nonempty, e0, e_end, carry):
    """(rows, seg0, carry) of the STEPS steps from e0, as the kernel's walk_rows."""
    rows, segs = [], []
    for k in range(STEPS):
        s0 = e0 + k * W
        if s0 >= e_end:
            rows.append([0] * W)
            segs.append([0] * W)
            continue
        mark = [-1] * W
        for r in range(W):
            rel = bnd[r] - s0
            if nonempty[r] and 0 <= rel < W:
                assert mark[rel] == -1  # one writer per position
                mark[rel] = (r << 6) | rel
        pk, run = [], -1
        for lane in range(W):
            run = max(run, mark[lane])
            pk.append(max(run, carry))
        carry = pk[W - 1] & ~63
        rows.append([p >> 6 for p in pk])
        segs.append([p & 63 for p in pk])
    return rows, segs, carry


def emulate(n, rp, col, lab, q):
    m = int(rp[-1])
    keep = np.full(m, 99, np.int64)
    deg = np.zeros(n, np.int64)
    for r0 in range(0, n, ROWS):
        xs = [min(r0 + lane, n) for lane in range(W)]
        bnd = [int(rp[xs[lane]]) if lane <= ROWS else 0 for lane in range(W)]
        row_ok = [lane < ROWS and r0 + lane < n for lane in range(W)]
        labv = [int(lab[r0 + lane]) if row_ok[lane] else 0 for lane in range(W)]
        cand = sum(1 << lane for lane in range(W) if row_ok[lane] and labv[lane] in q)
        nonempty = [row_ok[lane] and lane + 1 < W and bnd[lane + 1] > bnd[lane] for lane in range(W)]
        e_beg, e_end = bnd[0], bnd[ROWS]
        count = [0] * ROWS
        carry = -1
        e0 = e_beg
        while cand and e0 < e_end:
            rows, segs, carry = walk_rows(bnd, nonempty, e0, e_end, carry)
            for k in range(STEPS):
                kps = []
                for lane in range(W):
                    e = e0 + k * W + lane
                    act = e < e_end and (cand >> rows[k][lane]) & 1
                    if act:
                        assert bnd[rows[k][lane]] <= e < bnd[rows[k][lane] + 1]
                    kp = bool(act) and fits(q, labv[rows[k][lane]], int(lab[col[e]]))
                    if act:
                        keep[e] = kp
                    kps.append(kp)
                b = sum(1 << lane for lane in range(W) if kps[lane])
                for lane in range(W):
                    e = e0 + k * W + lane
                    nxt = lane + 1 < W and e + 1 < e_end and rows[k][lane + 1] == rows[k][lane]
                    if e < e_end and not nxt:
                        count[rows[k][lane]] += popc(b & lane_range(segs[k][lane], lane + 1))
            e0 += STEPS * W
        for lane in range(ROWS):
            if row_ok[lane]:
                deg[r0 + lane] = count[lane]
    off = np.concatenate([[0], np.cumsum(deg)])[:-1] if n else np.zeros(0, np.int64)
    kt = int(deg.sum())
    fcol = np.full(kt, -1, np.int64)
    for r0 in range(0, n, ROWS):
        xs = [min(r0 + lane, n) for lane in range(W)]
        bnd = [int(rp[xs[lane]]) if lane <= ROWS else 0 for lane in range(W)]
        row_ok = [lane < ROWS and r0 + lane < n for lane in range(W)]
        at = [(int(off[xs[lane]]) if xs[lane] < n else kt) if lane <= ROWS else 0
              for lane in range(W)]
        rowsm = sum(1 << lane for lane in range(W)
                    if row_ok[lane] and lane + 1 < W and at[lane + 1] > at[lane])
        nonempty = [row_ok[lane] and lane + 1 < W and bnd[lane + 1] > bnd[lane] for lane in range(W)]
        e_beg, e_end = bnd[0], bnd[ROWS]
        count = [0] * ROWS
        carry = -1
        e0 = e_beg
        while rowsm and e0 < e_end:
            rows, segs, carry = walk_rows(bnd, nonempty, e0, e_end, carry)
            for k in range(STEPS):
                kps = []
                for lane in range(W):
                    e = e0 + k * W + lane
                    kps.append(e < e_end and bool((rowsm >> rows[k][lane]) & 1) and keep[e] == 1)
                b = sum(1 << lane for lane in range(W) if kps[lane])
                for lane in range(W):
                    if kps[lane]:
                        r = rows[k][lane]
                        pos = at[r] + count[r] + popc(b & lane_range(segs[k][lane], lane))
                        assert 0 <= pos < kt and fcol[pos] == -1
                        fcol[pos] = col[e0 + k * W + lane]
                for lane in range(W):
                    e = e0 + k * W + lane
                    nxt = lane + 1 < W and e + 1 < e_end and rows[k][lane + 1] == rows[k][lane]
                    if e < e_end and not nxt:
                        count[rows[k][lane]] += popc(b & lane_range(segs[k][lane], lane + 1))
            e0 += STEPS * W
    return deg, fcol


@pytest.mark.parametrize("seed", range(4))
def test_label_filter_indexing(seed):
    rng = np.random.default_rng(seed)
    for _ in range(12):
        n = int(rng.integers(0, 160))
        degs = rng.choice([0, 0, 1, 2, 3, 15, 40, 70, 130, 300], size=n)
        rp = np.concatenate([[0], np.cumsum(degs)]).astype(np.int64)
        col = rng.integers(0, max(n, 1), size=int(rp[-1]))
        lab = rng.integers(0, 3, size=n)
        q = sorted(rng.integers(0, 3, size=3).tolist())
        deg, fcol = emulate(n, rp, col, lab, q)
        want_deg, want_cols = np.zeros(n, np.int64), []
        for u in range(n):
            ks = [int(col[e]) for e in range(rp[u], rp[u + 1])
                  if lab[u] in q and fits(q, int(lab[u]), int(lab[col[e]]))]
            want_deg[u] = len(ks)
            want_cols += ks
        np.testing.assert_array_equal(deg, want_deg)
        np.testing.assert_array_equal(fcol, np.array(want_cols, np.int64))
