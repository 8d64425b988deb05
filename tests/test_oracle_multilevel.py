"""Pins of the oracle's nested refinement with more than two levels (the
two-level coupling of Sec. II.B applied at every interface of a chain of
boxes, as in the paper's four- and five-level setups)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1710_02065_amd import workloads as W

CS2 = 1.0 / 3.0


def level_coords(M, l):
    """Physical (level-0) coordinates of every node of level l."""
    nx, ny, nz = M.grids[l].shape
    k = np.arange(M.grids[l].N)
    p = [(k % nx).astype(float), ((k // nx) % ny).astype(float), (k // (nx * ny)).astype(float)]
    for m in range(l - 1, -1, -1):  # map level m+1 coordinates to level m
        lo = M.pairs[m].lo
        p = [lo[a] + p[a] / 2.0 for a in range(3)]
    if M.d == 2:
        p[2] = 0.0 * p[2]
    return p


@pytest.mark.parametrize("q,shape,lo,hi", [(9, (48, 40, 1), (12, 9, 0), (30, 25, 0)),
                                           (19, (22, 20, 18), (6, 5, 5), (14, 13, 12))])
def test_two_levels_equal_refined_grid(q, shape, lo, hi):
    d = 2 if q == 9 else 3
    fs = tuple(2 * (hi[a] - lo[a]) + 1 if a < d else 1 for a in range(3))
    fc = W.random_state(shape, seed=1, d=d, u_amp=0.03, rho_amp=0.01, pi_amp=5e-4)
    ff = W.random_state(fs, seed=2, d=d, u_amp=0.03, rho_amp=0.01, pi_amp=5e-4)
    a = O.RefinedGrid(q, *shape, lo=lo, hi=hi, tau=0.57)
    a.init(0, *fc)
    a.init(1, *ff)
    a.step(5)
    b = O.MultiLevelGrid(q, *shape, boxes=[(lo, hi)], tau=0.57)
    b.init(0, *fc)
    b.init(1, *ff)
    b.step(5)
    assert np.array_equal(a.coarse.f, b.grids[0].f)
    assert np.array_equal(a.fine.f, b.grids[1].f)


def three_levels(q, **kw):
    if q == 9:
        return O.MultiLevelGrid(9, 48, 40, 1, boxes=[((10, 8, 0), (36, 30, 0)),
                                                     ((12, 10, 0), (34, 30, 0))], **kw)
    return O.MultiLevelGrid(q, 24, 22, 20, boxes=[((5, 5, 5), (17, 16, 15)),
                                                  ((6, 6, 6), (16, 15, 14))], **kw)


@pytest.mark.parametrize("q", [9, 19])
def test_three_level_roles_and_times(q):
    M = three_levels(q, tau=0.6)
    # the middle level carries a RING shell and its child's IMPORT / COVERED
    # nodes, disjoint
    mid_ring = M.ring[1] != 0
    mid_child = M.crole[1] != O.NORMAL
    assert mid_ring.any() and mid_child.any() and not (mid_ring & mid_child).any()
    assert not M.ring[0].any() and not (M.crole[2] != O.NORMAL).any()
    assert M.grids[2].g.tau == pytest.approx((4 * ((4 * 0.6 - 1) / 2) - 1) / 2)
    for l in range(3):
        M.init(l)
    M.step(3)
    assert [g.t for g in M.grids] == [3, 6, 12]


@pytest.mark.parametrize("q", [9, 19])
def test_three_level_uniform_flow_is_fixed_point(q):
    u0 = np.array([0.05, -0.02, 0.03 if q != 9 else 0.0])
    M = three_levels(q, tau=0.58)
    for l, g in enumerate(M.grids):
        M.init(l, np.full(g.N, 1.02), np.tile(u0[:, None], (1, g.N)))
    f0 = [g.f.copy() for g in M.grids]
    M.step(6)
    for g, f in zip(M.grids, f0):
        assert np.abs(g.f - f).max() < 1e-14


def test_shear_wave_across_two_nested_interfaces():
    """u_x = A sin(k y) decaying at nu k^2 through a level-0 grid, a level-1
    box and a level-2 box inside it: every level within 1e-3 of the decay
    solution, mass drift bounded."""
    n, tau, A, T = 64, 0.6, 1e-3, 200
    M = O.MultiLevelGrid(9, n, n, 1, boxes=[((8, 16, 0), (40, 48, 0)),
                                            ((16, 12, 0), (48, 52, 0))], tau=tau)
    k = 2 * math.pi / n
    for l, g in enumerate(M.grids):
        _, Y, _ = level_coords(M, l)
        u = np.zeros((3, g.N))
        u[0] = A * np.sin(k * Y)
        p = np.zeros((6, g.N))
        # the non-equilibrium stress scales with tau and the level's time step
        p[3] = -g.g.tau * CS2 * A * k * np.cos(k * Y) * 0.5 ** l
        M.init(l, np.ones(g.N), u, p)
    normal0 = M.crole[0] == O.NORMAL
    m0 = M.grids[0].moments()[0][normal0].sum()
    M.step(T)
    amp = A * math.exp(-CS2 * (tau - 0.5) * k * k * T)
    for l, g in enumerate(M.grids):
        _, Y, _ = level_coords(M, l)
        keep = (M.crole[l] == O.NORMAL) & (M.ring[l] == 0)
        uu = g.moments()[1][0]
        err = np.abs(uu - amp * np.sin(k * Y))[keep].max() / amp
        assert err < 1e-3, (l, err)
    drift = abs(M.grids[0].moments()[0][normal0].sum() - m0) / m0
    assert drift < 1e-6


def five_levels(q, **kw):
    """Level 0 and four nested boxes, each at least 4 nodes inside its
    parent (the jet setup of Sec. IV uses five levels)."""
    if q == 9:
        return O.MultiLevelGrid(9, 40, 36, 1, boxes=[((8, 8, 0), (30, 28, 0)),
                                                     ((8, 8, 0), (36, 32, 0)),
                                                     ((10, 10, 0), (46, 40, 0)),
                                                     ((12, 12, 0), (60, 48, 0))], **kw)
    return O.MultiLevelGrid(q, 20, 20, 20, boxes=[((4, 4, 4), (13, 13, 13)),
                                                  ((4, 4, 4), (14, 14, 14)),
                                                  ((4, 4, 4), (16, 16, 16)),
                                                  ((4, 4, 4), (20, 20, 20))], **kw)


@pytest.mark.parametrize("q", [9, 27])
def test_five_level_uniform_flow_is_fixed_point_and_times(q):
    u0 = np.array([0.04, -0.03, 0.02 if q != 9 else 0.0])
    M = five_levels(q, tau=0.56)
    assert M.nlevels == 5
    taus = [g.g.tau for g in M.grids]
    for a, b in zip(taus, taus[1:]):
        assert b == pytest.approx((4 * a - 1) / 2, abs=1e-14)
    for l, g in enumerate(M.grids):
        M.init(l, np.full(g.N, 0.99), np.tile(u0[:, None], (1, g.N)))
    f0 = [g.f.copy() for g in M.grids]
    M.step(2)
    assert [g.t for g in M.grids] == [2, 4, 8, 16, 32]
    for g, f in zip(M.grids, f0):
        assert np.abs(g.f - f).max() < 1e-14


def shear_wave_five_levels(tau_bump=0.0):
    """u_x = A sin(k y) through level 0 and four nested boxes (four
    interfaces in a chain): maximum error of each level against the decay
    solution A exp(-nu k^2 t) sin(k y), and the mass drift of level 0."""
    n, tau, A, T = 64, 0.6, 1e-3, 120
    M = O.MultiLevelGrid(9, n, n, 1, boxes=[((8, 16, 0), (40, 48, 0)),
                                            ((16, 12, 0), (48, 52, 0)),
                                            ((16, 16, 0), (48, 64, 0)),
                                            ((16, 16, 0), (48, 80, 0))], tau=tau)
    if tau_bump:
        M.grids[-1].g.tau += tau_bump
    k = 2 * math.pi / n
    for l, g in enumerate(M.grids):
        _, Y, _ = level_coords(M, l)
        u = np.zeros((3, g.N))
        u[0] = A * np.sin(k * Y)
        p = np.zeros((6, g.N))
        p[3] = -g.g.tau * CS2 * A * k * np.cos(k * Y) * 0.5 ** l
        M.init(l, np.ones(g.N), u, p)
    normal0 = M.crole[0] == O.NORMAL
    m0 = M.grids[0].moments()[0][normal0].sum()
    M.step(T)
    amp = A * math.exp(-CS2 * (tau - 0.5) * k * k * T)
    errs = []
    for l, g in enumerate(M.grids):
        _, Y, _ = level_coords(M, l)
        keep = (M.crole[l] == O.NORMAL) & (M.ring[l] == 0)
        errs.append(float(np.abs(g.moments()[1][0] - amp * np.sin(k * Y))[keep].max() / amp))
    drift = abs(M.grids[0].moments()[0][normal0].sum() - m0) / m0
    return errs, drift


def test_shear_wave_across_four_nested_interfaces():
    """Every level of a five-level chain within 2e-4 of the decay solution
    (measured 3.1e-5 at most); the viscosity cs^2 (tau_l - 1/2) dx_l^2 / dt_l
    is the same on every level only with tau_(l+1) = (4 tau_l - 1)/2, and an
    innermost tau off by 0.05 (2.1 -> 2.15) fails the bar (6.4e-4)."""
    errs, drift = shear_wave_five_levels()
    assert max(errs) < 2e-4, errs
    assert drift < 1e-6
    bad, _ = shear_wave_five_levels(tau_bump=0.05)
    assert bad[-1] > 2e-4, bad
