"""The LDS layout of the direct-to-LDS tile engine (csrc/tile_dma.hpp),
checked on the host for every shape the library instantiates: per K chunk,
the copies of all waves fill each LDS slot of the A and B stages exactly
once; the EPL elements one lane copies (16 bytes) are consecutive rows or
columns of one k row, aligned to EPL (so that, with row blocks that are
multiples of EPL, they are consecutive in global memory); and the operand
each lane reads for each matrix-core step (k row 4 kk + lk, row or column
of its 16-lane group) is the slot the copy of that element filled.  The
index arithmetic below restates the engine's; a shape change that breaks
one of these properties fails here before it reaches a GPU."""
import pytest

# (WM, WN, NB, KC, S, element bytes): FP64 and FP32 stage C, FP32 stage A
# (wide and narrow) and FP32 stage B (WM 2..5, wide and narrow)
SHAPES = ([(4, 2, 5, 32, 2, 8), (4, 2, 5, 16, 3, 4), (4, 2, 6, 16, 2, 4), (4, 2, 2, 16, 2, 4)]
          + [(wm, 2, nb, 16, 2, 4) for wm in (2, 3, 4, 5) for nb in (2, 6)])


def rot(k, w, bw):
    g = bw // 16
    return ((16 * (k % g) - (k * w) % bw) % bw + bw) % bw


@pytest.mark.parametrize("shape", SHAPES)
def test_copy_and_read_layout(shape):
    WM, WN, NB, KC, S, size = shape
    ROWS, COLS, NW = 32 * WM, 16 * NB * WN, WM * WN
    EPL = 16 // size
    PER = 64 * EPL
    BW = 32 if size == 8 else 64
    ACH, BCH = KC * ROWS, KC * COLS
    assert ACH % PER == 0 and BCH % PER == 0 and ROWS % 16 == 0 and COLS % 16 == 0
    NCA, NCB = ACH // PER, BCH // PER
    NC = NCA + NCB
    CPW, CMIN = -(-NC // NW), NC // NW
    assert KC % 4 == 0 and S >= 2 and CMIN >= 1 and CMIN * (S - 2) < 16
    filled = {"A": {}, "B": {}}
    for wave in range(NW):
        nmine = CPW if wave + NW * (CPW - 1) < NC else CPW - 1
        for j in range(nmine):
            c = wave + NW * j
            assert c < NC
            isb = c >= NCA
            cl = (c - NCA if isb else c) * PER
            width = COLS if isb else ROWS
            for lane in range(64):
                e = cl + lane * EPL
                k, pos = divmod(e, width)
                x = (pos - rot(k, width, BW)) % width
                assert x % EPL == 0 and x + EPL <= width
                for i in range(EPL):
                    slot = cl + lane * EPL + i
                    assert slot == k * width + (x + i + rot(k, width, BW)) % width
                    key = "B" if isb else "A"
                    assert slot not in filled[key], (shape, key, slot)
                    filled[key][slot] = (k, x + i)
    assert len(filled["A"]) == ACH and len(filled["B"]) == BCH
    # operand reads of the matrix-core steps
    for wave in range(NW):
        wm, wn = wave % WM, wave // WM
        for lane in range(64):
            lr, lk = lane & 15, lane >> 4
            ra, rbo = rot(lk, ROWS, BW), rot(lk, COLS, BW)
            a0o = lk * ROWS + (wm * 32 + lr + ra) % ROWS
            a1o = lk * ROWS + (wm * 32 + 16 + lr + ra) % ROWS
            for kk in range(KC // 4):
                k = 4 * kk + lk
                assert filled["A"][kk * 4 * ROWS + a0o] == (k, wm * 32 + lr)
                assert filled["A"][kk * 4 * ROWS + a1o] == (k, wm * 32 + 16 + lr)
                for cb in range(NB):
                    bo = lk * COLS + ((wn * NB + cb) * 16 + lr + rbo) % COLS
                    assert filled["B"][kk * 4 * COLS + bo] == (k, (wn * NB + cb) * 16 + lr)


def test_lds_budget_of_the_fp64_default():
    """The FP64 stage-C default (<4,2,5,32,2>) with the 3968-entry panel
    table stays within the 160 KB of LDS a workgroup may use."""
    WM, WN, NB, KC, S, size = SHAPES[0]
    stages = S * KC * (32 * WM + 16 * NB * WN) * size
    assert stages + 3968 * 4 + 4 <= 160 * 1024
