"""Host emulation of the DPP lane-move sequences the kernels use for wave scans and shifts
(GFX9 data-parallel primitives, 64-lane wave in four rows of 16): row_shr:n, row_bcast:15,
row_bcast:31 and wave_shr:1, with a row mask and bound_ctrl off, so a lane with no valid
source, or outside the row mask, keeps the `old` operand.  The checks pin the sequences
themselves: Kogge-Stone inside rows, then the two broadcasts, gives an inclusive scan for any
associative operator with identity `old`; wave_shr:1 with `old` = first gives the value of the
previous lane."""
import numpy as np
import pytest

ROW_SHR = {1: 0x111, 2: 0x112, 4: 0x114, 8: 0x118}
WAVE_SHR1, ROW_BCAST15, ROW_BCAST31 = 0x138, 0x142, 0x143


def update_dpp(old, x, ctrl, row_mask):
    out = []
    for lane in range(64):
        row, pos = divmod(lane, 16)
        if not (row_mask >> row) & 1:
            out.append(old)
            continue
        if 0x111 <= ctrl <= 0x11F:
            n = ctrl - 0x110
            out.append(x[lane - n] if pos >= n else old)
        elif ctrl == WAVE_SHR1:
            out.append(x[lane - 1] if lane >= 1 else old)
        elif ctrl == ROW_BCAST15:
            out.append(x[16 * row - 1] if row >= 1 else old)
        elif ctrl == ROW_BCAST31:
            out.append(x[31] if row >= 2 else old)
        else:
            raise ValueError(hex(ctrl))
    return out


def dpp_inclusive_scan(x, identity, op):
    steps = [(ROW_SHR[1], 0xF), (ROW_SHR[2], 0xF), (ROW_SHR[4], 0xF), (ROW_SHR[8], 0xF),
             (ROW_BCAST15, 0xA), (ROW_BCAST31, 0xC)]
    for ctrl, row_mask in steps:
        y = update_dpp(identity, x, ctrl, row_mask)
        x = [op(b, a) for a, b in zip(x, y)]  # earlier lanes on the left
    return x


@pytest.mark.parametrize("name,identity,op", [
    ("sum", 0, lambda a, b: a + b),
    ("max", -(1 << 31), max),
    ("min", (1 << 63) - 1, min),
    ("concat", "", lambda a, b: a + b),  # not commutative: checks the operand order
])
def test_scan_sequence_is_an_inclusive_scan(name, identity, op):
    rng = np.random.default_rng(11)
    for _ in range(200):
        if name == "concat":
            x = [chr(65 + i % 26) + str(i) for i in range(64)]
        else:
            x = [int(v) for v in rng.integers(-5, 100, size=64)]
        got = dpp_inclusive_scan(list(x), identity, op)
        acc, want = identity, []
        for v in x:
            acc = op(acc, v)
            want.append(acc)
        assert got == want


def test_wave_shift_gives_previous_lane():
    x = list(range(100, 164))
    got = update_dpp(-7, x, WAVE_SHR1, 0xF)
    assert got == [-7] + x[:-1]


def test_row_shift_does_not_cross_rows():
    x = list(range(64))
    got = update_dpp(-1, x, ROW_SHR[1], 0xF)
    assert [got[16 * r] for r in range(4)] == [-1] * 4
    assert got[17] == 16
