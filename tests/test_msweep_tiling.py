"""Host-side model of the moment sweep's work decomposition (CPU).

k_msweep gives each workgroup a TX x TY tile of a plane plus a one-cell
halo and a chunk of planes.  In 3D the wavefronts split the halo plane by
role: TY interior wavefronts (lane = x, wavefront = y of the output cell,
which is also the slot rebuilt), one per halo row (only the populations
with xi_y = +1 below the tile, -1 above it) and one for both halo columns
(only xi_x != 0); interior cells take the populations with no in-plane
velocity from their own registers.  In 2D each thread owns one slot of the
halo row.  This model replays the kernel's index arithmetic (tile
constants read from the source) for ragged and degenerate grids and checks
that every load and store is in bounds, every cell is written exactly once
per step, no (direction, slot) pair is written twice, every slot read for
direction i was written for direction i in the same plane, and it holds
the source cell x - xi under periodic wrap.
"""
import itertools
import os
import re

import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1710_02065_amd", "csrc", "msweep.hip")


def tile_constants():
    s = open(SRC).read()
    tx = re.search(r"TX = L::D == 3 \? (\d+) : (\d+);", s)
    ty = re.search(r"TY = L::D == 3 \? \(sizeof\(R\) == 8 \? (\d+) : (\d+)\) : 1;", s)
    assert tx and ty, "tile constants not found in msweep.hip"
    return dict(tx3=int(tx.group(1)), tx2=int(tx.group(2)), ty64=int(ty.group(1)),
                ty32=int(ty.group(2)))


def directions(q):
    if q == 9:
        return [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (1, 1, 0), (-1, -1, 0),
                (1, -1, 0), (-1, 1, 0)]
    out = []
    for d in itertools.product((-1, 0, 1), repeat=3):
        s = sum(abs(x) for x in d)
        if q == 19 and s == 3:
            continue
        out.append(d)
    return out


def replay(q, shape, fp64, block, k):
    D = 2 if q == 9 else 3
    TX = k["tx3"] if D == 3 else k["tx2"]
    TY = (k["ty64"] if fp64 else k["ty32"]) if D == 3 else 1
    HX, HY = TX + 2, (TY + 2 if D == 3 else 1)
    SLOTS = HX * HY
    NT = (TY + 3) * 64 if D == 3 else (SLOTS + 63) // 64 * 64
    if D == 3:
        assert TX == 64 and 2 * HY <= 64
    nx, ny, nz = shape
    px, py, pm = nx, (ny if D == 3 else 1), (nz if D == 3 else ny)
    N = nx * ny * nz
    tiles_x, tiles_y = -(-px // TX), -(-py // TY)
    zc = min(64, max(4, block // 16))
    chunks = -(-pm // zc)
    nb = tiles_x * tiles_y * chunks
    xcd = nb % 8 == 0
    dv = directions(q)
    Q = len(dv)
    shift = [d[0] + (d[1] * HX if D == 3 else 0) for d in dv]
    written = np.zeros(N, dtype=np.int64)
    tiles = set()
    tid = np.arange(NT)
    wave, lane = tid // 64, tid % 64
    for blk in range(nb):
        b = (blk % 8) * (nb // 8) + blk // 8 if xcd else blk
        tiles.add(b)
        bx, r = b % tiles_x, b // tiles_x
        by, ch = r % tiles_y, r // tiles_y
        x0, y0 = bx * TX, by * TY
        wx, wy = min(TX, px - x0), (min(TY, py - y0) if D == 3 else 1)
        m0 = ch * zc
        m1 = min(pm, m0 + zc)
        plane = px * py
        # per thread: slot (sx, sy), the plane cell it loads, whether it
        # writes the slot, and which directions it writes
        needs = np.zeros((NT, Q), dtype=bool)
        if D == 3:
            hy = wy + 2
            sx = np.zeros(NT, dtype=np.int64)
            sy = np.zeros(NT, dtype=np.int64)
            gx = np.zeros(NT, dtype=np.int64)
            gy = np.zeros(NT, dtype=np.int64)
            sown = np.zeros(NT, dtype=bool)
            inner = wave < TY
            oxc, oyc = np.minimum(lane, wx - 1), np.minimum(wave, wy - 1)
            sx[inner], sy[inner] = oxc[inner] + 1, oyc[inner] + 1
            gx[inner], gy[inner] = x0 + oxc[inner], y0 + oyc[inner]
            sown[inner] = ((lane < wx) & (wave < wy))[inner]
            for i, d in enumerate(dv):
                needs[inner, i] = shift[i] != 0
            for w, lo in ((TY, True), (TY + 1, False)):
                rw = wave == w
                sx[rw] = np.minimum(lane[rw], wx - 1) + 1
                sy[rw] = 0 if lo else wy + 1
                gx[rw] = x0 + sx[rw] - 1
                gy[rw] = (y0 + py - 1) % py if lo else (y0 + wy) % py
                sown[rw] = lane[rw] < wx
                for i, d in enumerate(dv):
                    needs[rw, i] = d[1] == (1 if lo else -1)
            cw = wave == TY + 2
            left = lane < hy
            csy = np.where(left, lane, np.minimum(lane - hy, hy - 1))
            sx[cw] = np.where(left, 0, wx + 1)[cw]
            sy[cw] = csy[cw]
            gx[cw] = np.where(left, (x0 + px - 1) % px, (x0 + wx) % px)[cw]
            gy[cw] = ((y0 + csy + py - 1) % py)[cw]
            sown[cw] = (lane < 2 * hy)[cw]
            for i, d in enumerate(dv):
                needs[cw, i] = d[0] != 0
            assert gx.min() >= 0 and gx.max() < px and gy.min() >= 0 and gy.max() < py
            scell = gy * px + gx
        else:
            hx = wx + 2
            sown = tid < hx
            sx = np.where(sown, tid, 0)
            sy = np.zeros_like(sx)
            scell = (x0 + sx + px - 1) % px
            needs[:] = True
        slds = sy * HX + sx
        assert slds[sown].max() < SLOTS
        # slot_cell[i, s]: the cell whose direction-i population slot s holds
        slot_cell = np.full((Q, SLOTS), -1)
        for i in range(Q):
            wr = sown & needs[:, i]
            assert len(set(slds[wr])) == int(wr.sum()), "slot written twice"
            slot_cell[i, slds[wr]] = scell[wr]
        # loads: planes m0 - 1 ... m1 + 1, wrapped
        for m in range(m0 - 1, m1 + 2):
            c = ((m + pm) % pm) * plane + scell
            assert c.min() >= 0 and c.max() < N
        if D == 3:
            ox, oy = lane, wave
            oown = (wave < TY) & (ox < wx) & (oy < wy)
            # an interior thread's own slot is its output cell
            assert np.array_equal(scell[oown], ((y0 + oy) * px + x0 + ox)[oown])
        else:
            ox, oy = tid, np.zeros_like(tid)
            oown = tid < wx
        ocell = (y0 + oy) * px + x0 + ox
        olds = ((oy + 1) * HX if D == 3 else 0) + ox + 1
        for i, d in enumerate(dv):
            ex = (x0 + ox[oown] - d[0]) % px
            ey = ((y0 + oy[oown] - d[1]) % py) if D == 3 else np.zeros_like(ex)
            if D == 3 and shift[i] == 0:
                src = scell[oown]  # from the thread's own registers
            else:
                li = olds[oown] - shift[i]
                assert li.min() >= 0 and li.max() < SLOTS
                src = slot_cell[i, li]
                assert src.min() >= 0, "read of a slot no thread wrote"
            np.testing.assert_array_equal(src, ey * px + ex)
        for m in range(m0, m1):
            c = m * plane + ocell[oown]
            assert c.min() >= 0 and c.max() < N
            np.add.at(written, c, 1)
    assert len(tiles) == nb
    assert written.min() == 1 and written.max() == 1


SHAPES = [(9, (300, 37, 1)), (9, (1, 1, 1)), (9, (1, 5, 1)), (9, (7, 1, 1)), (9, (255, 3, 1)),
          (19, (150, 13, 37)), (19, (1, 1, 1)), (19, (2, 3, 1)), (19, (65, 5, 2)),
          (19, (64, 16, 40)), (27, (70, 11, 21)), (27, (3, 1, 2)), (27, (1, 9, 1)),
          (27, (40, 9, 12))]


@pytest.mark.parametrize("q,shape", SHAPES)
@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("block", [64, 256, 1024])
def test_msweep_decomposition(q, shape, fp64, block):
    replay(q, shape, fp64, block, tile_constants())


def test_msweep_decomposition_headline_launch():
    """D3Q19 256^3 FP32 with 64 planes per workgroup, the configuration the
    benchmark times (512 workgroups, XCD-ordered)."""
    replay(19, (256, 256, 256), False, 1024, tile_constants())
