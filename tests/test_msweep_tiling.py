"""Host-side model of the moment sweep's work decomposition (CPU).

k_msweep gives each workgroup a TX x TY tile of a plane plus a one-cell
halo and a chunk of planes; threads own halo-plane slots, and interior
threads pull population i of their cell from the slot at x - xi.  This
model replays the kernel's index arithmetic (tile constants read from the
source) for ragged and degenerate grids and checks that every load and
store is in bounds, every cell is written exactly once per step, every
slot read was written in the same plane, and the slot read for direction i
holds the source cell x - xi under periodic wrap.
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
    NT = (SLOTS + 63) // 64 * 64
    nx, ny, nz = shape
    px, py, pm = nx, (ny if D == 3 else 1), (nz if D == 3 else ny)
    N = nx * ny * nz
    tiles_x, tiles_y = -(-px // TX), -(-py // TY)
    zc = min(64, max(4, block // 16))
    chunks = -(-pm // zc)
    nb = tiles_x * tiles_y * chunks
    xcd = nb % 8 == 0
    dv = directions(q)
    shift = [d[0] + (d[1] * HX if D == 3 else 0) for d in dv]
    written = np.zeros(N, dtype=np.int64)
    tiles = set()
    tid = np.arange(NT)
    for blk in range(nb):
        b = (blk % 8) * (nb // 8) + blk // 8 if xcd else blk
        tiles.add(b)
        bx, r = b % tiles_x, b // tiles_x
        by, ch = r % tiles_y, r // tiles_y
        x0, y0 = bx * TX, by * TY
        wx, wy = min(TX, px - x0), (min(TY, py - y0) if D == 3 else 1)
        m0 = ch * zc
        m1 = min(pm, m0 + zc)
        hx, hy = wx + 2, (wy + 2 if D == 3 else 1)
        plane = px * py
        sown = tid < hx * hy
        sx = np.where(sown, tid % hx, 0)
        sy = np.where(sown, tid // hx, 0)
        gx = (x0 + sx + px - 1) % px
        gy = (y0 + sy + py - 1) % py if D == 3 else np.zeros_like(sx)
        scell = gy * px + gx
        slds = sy * HX + sx
        assert slds[sown].max() < SLOTS and len(set(slds[sown])) == int(sown.sum())
        slot_cell = np.full(SLOTS, -1)
        slot_cell[slds[sown]] = scell[sown]
        # loads: planes m0 - 1 ... m1 + 1, wrapped
        for m in range(m0 - 1, m1 + 2):
            c = ((m + pm) % pm) * plane + scell
            assert c.min() >= 0 and c.max() < N
        ox, oy = tid % TX, tid // TX
        oown = (tid < TX * TY) & (ox < wx) & (oy < wy)
        ocell = (y0 + oy) * px + x0 + ox
        olds = ((oy + 1) * HX if D == 3 else 0) + ox + 1
        for i, d in enumerate(dv):
            li = olds[oown] - shift[i]
            assert li.min() >= 0 and li.max() < SLOTS
            src = slot_cell[li]
            assert src.min() >= 0, "read of a slot no thread wrote"
            ex = (x0 + ox[oown] - d[0]) % px
            ey = ((y0 + oy[oown] - d[1]) % py) if D == 3 else np.zeros_like(ex)
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
