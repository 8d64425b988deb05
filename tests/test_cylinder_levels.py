"""Host-side geometry of the nested-level cylinder study (no GPU)."""
import pytest

from paper_1710_02065_amd import cylinder_levels as C
from paper_1710_02065_amd import lbm


@pytest.mark.parametrize("levels,D", [(4, 32), (3, 16), (2, 8)])
def test_boxes_nest_and_validate(levels, D):
    hw = (24.0, 10.0, 4.0)[: levels - 1]
    n0, D0, boxes, centres = C.geometry(levels, D, 160.0, hw, 1.5)
    assert D0 * 2 ** (levels - 1) == D
    # the body centre maps through every interface: x_child = 2 (x_parent - lo)
    for l, (lo, hi) in enumerate(boxes):
        cp, cc = centres[l], centres[l + 1]
        assert cc == (2 * (cp[0] - lo[0]), 2 * (cp[1] - lo[1]))
        # the body (radius D/2 on the finest level) stays inside every box
        r = D0 * 2 ** l / 2.0
        assert lo[0] + 4 <= cp[0] - r and cp[0] + r <= hi[0] - 4
        assert lo[1] + 4 <= cp[1] - r and cp[1] + r <= hi[1] - 4
    cfg = lbm.make_config(lattice=9, shape=(n0, n0, 1), tau=0.51, storage="f32", ma=0.2,
                          face_bc=(2, 2, 2, 2, 0, 0), refine_lo=boxes[0][0],
                          refine_hi=boxes[0][1], nest=tuple(boxes[1:]),
                          flags=lbm.LBM_SPONGE_FIELD)
    assert lbm.lbm_required_bytes(cfg) > 0, lbm.lbm_last_error()


def test_level_zero_needs_two_cells_per_diameter():
    with pytest.raises(ValueError):
        C.geometry(4, 8, 160.0, (24.0, 10.0, 4.0), 1.5)
    with pytest.raises(ValueError):
        C.geometry(4, 36, 160.0, (24.0, 10.0, 4.0), 1.5)


def test_relaxation_times_follow_the_interface_rule():
    t = C._taus(0.51, 4)
    for a, b in zip(t, t[1:]):
        assert abs(b - (2 * a - 0.5)) < 1e-15


def test_locate_maps_points_to_the_finest_level_holding_them():
    import numpy as np
    n0, D0, boxes, centres = C.geometry(4, 32, 160.0, (24.0, 10.0, 4.0), 1.5)
    shapes = [(n0, n0)]
    for lo, hi in boxes:
        shapes.append((2 * (hi[0] - lo[0]) + 1, 2 * (hi[1] - lo[1]) + 1))
    c = centres[0]
    r = np.geomspace(2.0 * D0, 45.0 * D0, 20)
    lev, cells = C.locate(np.stack([np.full_like(r, c[0]), c[1] + r], 1), boxes, shapes)
    assert lev[0] == 3 and lev[-1] == 0 and np.all(np.diff(lev) <= 0)
    for l, cell, rr in zip(lev, cells, r):
        nx = shapes[l][0]
        x, y = float(cell % nx), float(cell // nx)
        for k in range(l, 0, -1):
            lo = boxes[k - 1][0]
            x, y = x / 2 + lo[0], y / 2 + lo[1]
        assert abs(x - c[0]) <= 0.5 and abs(y - (c[1] + rr)) <= 0.5
