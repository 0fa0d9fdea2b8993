"""Geometry of the fused matrix-core tile (CPU only): for every tile shape the
library instantiates and every radius it sends there, a model of the
kernel's chunk, fragment and wave assignments checks that
* each output's band of 2W+1 taps lies inside the chunks its MFMAs read, in
  both passes, and every chunk a block skips holds only zero taps for it;
* the halo rows and columns a tile needs lie inside what it loads (32Q rows)
  and what its column-pass waves compute (16 kNCW columns), and the row pass
  reads no column those waves leave unwritten;
* fragment indices and tap-table indices stay in range;
* LDS offsets stay inside one buffer.
The model restates the kernel's index arithmetic (FusedTile in device.hpp)."""
import pytest

TAB_PAD = 32


def geometries():
    # (NW, TR, TC, Q, W range) as the single-image forward (FP16 / BF16), the
    # batched, pivoted and joint kernels use them
    out = []
    for nw, tr, tc, q, wlo, whi in ((8, 64, 64, 3, 1, 16), (8, 64, 64, 4, 17, 32), (8, 64, 32, 5, 33, 48),
                                    (16, 64, 128, 3, 1, 16), (16, 64, 128, 4, 17, 32), (16, 64, 64, 5, 33, 48),
                                    (16, 32, 128, 5, 49, 64)):
        for W in range(wlo, whi + 1):
            out.append((nw, tr, tc, q, W))
    return out


@pytest.mark.parametrize("NW,TR,TC,Q,W", geometries())
def test_tile_geometry(NW, TR, TC, Q, W):
    QA = (2 * W + 15) // 32
    QB = Q - TR // 32
    NRB, NCB = TR // 16, TC // 16
    WPR = NW // NRB
    JB = NCB // WPR
    NCW = NCB + 2 * QB
    pitch = 2 * (8 * NCW + (6 - 8 * NCW) % 32)
    assert pitch >= 16 * NCW and (pitch // 2) % 32 == 6 and pitch % 2 == 0
    assert QA in (QB - 1, QB)
    assert JB in (1, 2) and NCB % WPR == 0
    assert NCW <= NW
    assert TR + 2 * W <= 32 * Q, "halo rows loaded"
    assert TC + 2 * W <= 16 * NCW, "halo columns computed"
    tab_len = TAB_PAD + 32 * Q

    def tap(t):
        return 0 <= t <= 2 * W

    # column pass: block j, chunks q in [j/2, min(Q-1, j/2 + (QB if odd else QA))]
    for j in range(NRB):
        qs = range(j // 2, min(Q - 1, j // 2 + (QB if j & 1 else QA)) + 1)
        for q in range(Q):
            for i in range(16):                   # output row 16 j + i (tile-relative)
                for k in range(32):               # halo row 32 q + k
                    t = 32 * q + k - 16 * j - i   # tap index of that halo row for this output
                    if q not in qs:
                        assert not tap(t), (j, q, i, k)
                    # fragment tf[2q - j + 1]: element (li = i, k) is w[16 d + k - i], d = 2q - j
            if q in qs:
                assert 0 <= 2 * q - j + 1 < 2 * Q
        for i in range(16):
            need = set(range(16 * j + i, 16 * j + i + 2 * W + 1))
            have = set(r for q in qs for r in range(32 * q, 32 * q + 32))
            assert need <= have, (j, i)
    # tap table reads: kTabPad + 16 d + 8 lg + jj - li for d in [-1, 2Q-2]
    for d in range(-1, 2 * Q - 1):
        for lg in range(4):
            for jj in range(8):
                for li in range(16):
                    idx = TAB_PAD + 16 * d + 8 * lg + jj - li
                    assert 0 <= idx < tab_len
    # row pass: wave -> (rb, p); JB = 2: blocks 2p, 2p+1 from chunk base 32p;
    # JB = 1: block p from chunk base 32 (p // 2), fragments by the parity of p
    for wave in range(NW):
        rb, p = divmod(wave, WPR)
        assert rb < NRB
        blocks = [2 * p, 2 * p + 1] if JB == 2 else [p]
        for jc in blocks:
            base = 32 * p if JB == 2 else 32 * (p // 2)
            odd = jc & 1
            qs = range(QB + 1) if odd else range(QA + 1)
            frag = (lambda q: 2 * q) if odd else (lambda q: 2 * q + 1)
            for q in qs:
                assert 0 <= frag(q) < 2 * Q
                # column reads of ld_frag: 8 lg + [0, 8) within the chunk, 4 lg values of li rows
                assert base + 32 * q + 31 < 16 * NCW, "row pass reads an unwritten column"
                assert (16 * rb + 15) * pitch + 8 * 3 + base + 32 * q + 7 < TR * pitch
            for i in range(16):                   # output column 16 jc + i
                c = 16 * jc + i
                need = set(range(c, c + 2 * W + 1))
                have = set(col for q in qs for col in range(base + 32 * q, base + 32 * q + 32))
                assert need <= have, (wave, jc, i)
                # chunks the block does not read hold no tap for it
                for q in range(2 * Q):
                    if q in qs:
                        continue
                    for k in range(32):
                        assert not tap(base + 32 * q + k - c)
    # column pass LDS writes: row 16 j + li, column 16 wave + 4 lg + v
    assert (16 * (NRB - 1) + 15) * pitch + 16 * (NCW - 1) + 4 * 3 + 3 < TR * pitch


def _strip_length(tiles_x, tiles_y, cus):
    # the launcher's choice: the longest strip among those with the fewest tile rounds
    best, length = None, 1
    for L in range(1, tiles_y + 1):
        strips = tiles_x * -(-tiles_y // L)
        rounds = -(-strips // cus) * L
        if best is None or rounds <= best:
            best, length = rounds, L
    return length


@pytest.mark.parametrize("H,Wd,cus", [(4096, 4096, 256), (4000, 2100, 256), (1100, 4200, 256), (64, 128, 256),
                                      (4096, 4096, 304), (3000, 3000, 80), (700, 130, 7), (4096, 512, 256)])
def test_strip_order_covers_every_tile_once(H, Wd, cus):
    """Strips of the single-image FP16 kernel (64 x 128 tiles): the XCD-aware
    order of blocks (block b to XCD b mod 8, each XCD a contiguous range of
    strips in row-major order) gives every tile to exactly one block, and
    each block's tiles form one column, top to bottom."""
    tiles_x, tiles_y = -(-Wd // 128), -(-H // 64)
    L = _strip_length(tiles_x, tiles_y, cus)
    G = tiles_x * -(-tiles_y // L)
    gq, gr = G // 8, G % 8
    owner = {}
    for b in range(G):
        x = b % 8
        strip = x * gq + min(x, gr) + b // 8
        assert 0 <= strip < G
        cx, ty0 = strip % tiles_x, (strip // tiles_x) * L
        for ty in range(ty0, min(ty0 + L, tiles_y)):
            assert (ty, cx) not in owner
            owner[(ty, cx)] = b
    assert len(owner) == tiles_x * tiles_y
    if tiles_x * tiles_y > cus:
        assert L >= 1 and -(-G // cus) * L <= -(-(tiles_x * tiles_y) // cus)
