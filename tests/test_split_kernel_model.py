"""CPU model of the data movement of the split-form second contraction kernel.

The one-workgroup-per-CU kernel moves operands global -> LDS with 16-byte
direct loads (lane L of a wave writes LDS bytes [16 L, 16 L + 16) of its 1 KB
block) into a ring of three stages, reads them back LDS -> registers in the
matrix-core operand layout, clamps rows past M or N and K tiles past the range,
and renumbers blocks so that each XCD takes a contiguous run.  This model
restates those index rules (tile 256 x 128, four waves of 128 x 64, K tile 16,
four 16-bit planes) and checks, over tiny, ragged, multi-tile and split-K
shapes of K-blocked panels:

* every global element a direct load reads lies inside its plane;
* every LDS byte written or read lies inside its stage and operand region;
* every register operand equals the expected (plane, row, k) at every K tile,
  through the stage rotation (so no stage is overwritten before it is read);
* each 16-lane phase of an operand read touches 16 different bank groups;
* the XCD renumbering is a bijection of the launch.
"""

import numpy as np
import pytest

TM, TN = 256, 128
APLANE, BPLANE = TM * 32, TN * 32
STAGE = 4 * APLANE + 4 * BPLANE
LDS = 3 * STAGE
DA, DB = 4 * TM // 32 // 4, 4 * TN // 32 // 4


def pad_kt(v):
    return (v + 15) // 16 * 16


def code(plane, row, k):
    return (plane << 40) | (row << 20) | k


def panel(rows, K):
    """Four planes of codes in the K-blocked layout: (r, k) at (k // 16) * rows * 16 + r * 16 + k % 16."""
    ps = rows * K
    buf = np.full(4 * ps, -1, dtype=np.int64)
    r = np.arange(rows)[:, None]
    k = np.arange(K)[None, :]
    for p in range(4):
        buf[p * ps + (k // 16) * rows * 16 + r * 16 + k % 16] = code(p, r, k)
    return buf, ps


def xcd_run_index(b, total):
    x, idx = b % 8, b // 8
    return x * (total // 8) + min(x, total % 8) + idx


def simulate(M, N, K, split):
    A, aps = panel(M, K)
    B, bps = panel(N, K)
    lda, ldb = M * 16, N * 16
    tiles_n = (N + TN - 1) // TN
    count = ((M + TM - 1) // TM) * tiles_n
    total = count * split
    chunk = pad_kt((K + split - 1) // split)
    lane = np.arange(64)
    lr = lane >> 1
    lh = (lane & 1) ^ ((lr >> 3) & 1)
    l32, g = lane & 31, lane >> 5
    slot = (2 * l32 + (g ^ ((l32 >> 3) & 1))) * 16
    checked = 0
    for blk_id in range(total):
        bid = xcd_run_index(blk_id, total)
        s, t = divmod(bid, count)
        m0, n0 = (t // tiles_n) * TM, (t % tiles_n) * TN
        kb = s * chunk
        ke = min(K, kb + chunk)
        nk = (ke - kb) // 16 if ke > kb else 0
        if nk == 0:
            continue
        lds = np.full(LDS // 2, -7, dtype=np.int64)  # one cell per 16-bit element

        def issue(kt, so):
            tt = min(kt, nk - 1)
            for w in range(4):
                for u in range(DA):
                    blk = w + 4 * u
                    plane, rb = blk // 8, blk % 8
                    m = np.minimum(m0 + 32 * rb + lr, M - 1)
                    byte = (((kb >> 4) * lda + m0 * 16) * 2 + tt * lda * 2 + plane * aps * 2
                            + ((m - m0) * 16 + 8 * lh) * 2)
                    el = byte // 2
                    assert np.all(el >= plane * aps) and np.all(el + 8 <= (plane + 1) * aps)
                    dst = so + blk * 1024 + lane * 16
                    assert np.all(dst >= so) and np.all(dst + 16 <= so + 4 * APLANE)
                    for q in range(8):
                        lds[dst // 2 + q] = A[el + q]
                for u in range(DB):
                    blk = w + 4 * u
                    plane, rb = blk // 4, blk % 4
                    n = np.minimum(n0 + 32 * rb + lr, N - 1)
                    byte = (((kb >> 4) * ldb + n0 * 16) * 2 + tt * ldb * 2 + plane * bps * 2
                            + ((n - n0) * 16 + 8 * lh) * 2)
                    el = byte // 2
                    assert np.all(el >= plane * bps) and np.all(el + 8 <= (plane + 1) * bps)
                    dst = so + 4 * APLANE + blk * 1024 + lane * 16
                    assert np.all(dst + 16 <= so + STAGE)
                    for q in range(8):
                        lds[dst // 2 + q] = B[el + q]

        def check_registers(so, kt):
            for w in range(4):
                wm, wn = (w >> 1) * 128, (w & 1) * 64
                for i in range(4):
                    row = np.minimum(m0 + wm + 32 * i + l32, M - 1)
                    for c in range(4):
                        ad = so + (wm >> 5) * 1024 + slot + c * APLANE + i * 1024
                        assert np.all(ad >= so) and np.all(ad + 16 <= so + 4 * APLANE)
                        for q in range(8):
                            want = code(c, row, kb + 16 * kt + 8 * g + q)
                            assert np.all(lds[ad // 2 + q] == want)
                for j in range(2):
                    row = np.minimum(n0 + wn + 32 * j + l32, N - 1)
                    for c in range(4):
                        ad = so + 4 * APLANE + (wn >> 5) * 1024 + slot + c * BPLANE + j * 1024
                        assert np.all(ad + 16 <= so + STAGE)
                        for q in range(8):
                            want = code(c, row, kb + 16 * kt + 8 * g + q)
                            assert np.all(lds[ad // 2 + q] == want)

        # prologue: K tiles 0, 1, 2 into stages 0, 1, 2; registers <- tile 0
        issue(0, 0)
        issue(1, STAGE)
        issue(2, 2 * STAGE)
        check_registers(0, 0)
        cur, nxt, far = 0, STAGE, 2 * STAGE
        for kt in range(nk):
            # after the barrier of K tile kt: tile kt + 3 into the stage of tile kt,
            # then tile kt + 1 read from its stage
            issue(kt + 3, cur)
            if kt + 1 < nk:
                check_registers(nxt, kt + 1)
            cur, nxt, far = nxt, far, cur
            checked += 1
    return checked


@pytest.mark.parametrize("M,N,K,split", [(128, 128, 80, 2), (72, 136, 112, 3), (512, 256, 144, 2),
                                         (40, 24, 48, 1), (264, 200, 96, 4)])
def test_split_kernel_data_movement(M, N, K, split):
    assert simulate(M, N, K, split) > 0


def test_operand_reads_are_bank_conflict_free():
    for g in range(2):
        for half in range(2):
            l32 = np.arange(16 * half, 16 * half + 16)
            groups = (2 * l32 + (g ^ ((l32 >> 3) & 1))) % 16
            assert len(set(groups.tolist())) == 16


@pytest.mark.parametrize("total", list(range(1, 70)) + [256, 511, 4097])
def test_xcd_renumbering_is_a_bijection(total):
    assert sorted(xcd_run_index(b, total) for b in range(total)) == list(range(total))


def band_tile(local, tiles_m, tiles_n, rows=8):
    """The single-problem direct schedule's band order (ntgemm.hip, band_tile)."""
    band = local // (rows * tiles_n)
    h = min(rows, tiles_m - band * rows)
    r = local - band * rows * tiles_n
    return band * rows + r % h, r // h


@pytest.mark.parametrize("tiles_m,tiles_n", [(16, 32), (1, 1), (3, 5), (8, 16), (17, 9), (128, 128)])
def test_band_order_is_a_bijection_and_xcd_runs_are_compact(tiles_m, tiles_n):
    count = tiles_m * tiles_n
    tiles = [band_tile(t, tiles_m, tiles_n) for t in range(count)]
    assert sorted(tiles) == [(m, n) for m in range(tiles_m) for n in range(tiles_n)]
    if (tiles_m, tiles_n) == (16, 32):
        # 512 tiles of the 2048^2 FP32 second contraction: every XCD an 8 x 8 block
        for x in range(8):
            run = {tiles[xcd_run_index(b, count)] for b in range(count) if b % 8 == x}
            assert len({m for m, _ in run}) == 8 and len({n for _, n in run}) == 8
