"""Pins of the comparator operators the paper measures the regularized
collision against (Sec. II.A): LBM-BGK (eq. standardLB) and LBM-MRT on
D2Q9 (Lallemand & Luo 2000)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1710_02065_amd import workloads as W

CS2 = 1.0 / 3.0


def rand_f(seed):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.1, 0.1, 3)
    u[2] = 0.0
    f = O.equilibrium(9, rng.uniform(0.95, 1.05), u)
    return f + 2e-3 * rng.normal(size=9) * f


@pytest.mark.parametrize("tau", [0.52, 0.6, 1.3])
def test_mrt_with_equal_rates_is_bgk(tau):
    for seed in range(5):
        f = rand_f(seed)
        a = O.collide_mrt(f, [1 / tau] * 4)
        b = O.collide_bgk(9, f, tau)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_mrt_conserves_and_keeps_equilibrium():
    xi, _, _ = O.lattice(9)
    rates = [1.64, 1.54, 1.9, 1 / 0.57]
    for seed in range(5):
        f = rand_f(seed)
        p = O.collide_mrt(f, rates)
        assert p.sum() == pytest.approx(f.sum(), abs=1e-15)
        np.testing.assert_allclose(p @ xi, f @ xi, atol=1e-16)
        # the second-order equilibrium (the BGK one) is a fixed point
        rho, j = f.sum(), f @ xi
        u = j / rho
        feq = np.array([w * rho * (1 + 3 * (x @ u) + 4.5 * (x @ u) ** 2 - 1.5 * (u @ u))
                        for x, w in zip(xi.astype(float), O.lattice(9)[1])])
        np.testing.assert_allclose(O.collide_mrt(feq, rates), feq, atol=1e-16)


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_comparator_grid_viscosity_and_conservation(collision):
    """Taylor-Green decay on D2Q9 128^2: nu = cs^2 (tau - 1/2) within 5e-3
    (for MRT the shear viscosity follows s_nu = 1/tau alone); mass and
    momentum conserved to rounding."""
    n, U, tau = 64, 0.03, 0.6
    rho, u, _ = W.taylor_green_2d(n, U)
    g = O.Grid(9, n, n, 1, tau=tau, collision=collision).init(rho, u)
    mode = W.taylor_green_mode_2d(n)
    m0 = g.f.sum()
    g.step(50)
    a0 = g.moments()[1][0] @ mode / (mode @ mode)
    T = 600
    g.step(T)
    r, uu = g.moments()
    a1 = uu[0] @ mode / (mode @ mode)
    k = 2 * math.pi / n
    nu = -math.log(a1 / a0) / (2 * k * k * T)
    assert nu == pytest.approx(CS2 * (tau - 0.5), rel=5e-3)
    assert abs(g.f.sum() - m0) < 1e-12 * m0


def advected_shear_rate(collision, U, n=64, tau=0.6, steps=400):
    rho, u = W.shear_wave(n, 1, 1, 1e-3, advect=(U, 0.0, 0.0))
    g = O.Grid(9, n, 1, 1, tau=tau, collision=collision).init(rho, u)
    g.step(50)
    a0 = abs(np.fft.fft(g.moments()[1][1])[1])
    g.step(steps)
    a1 = abs(np.fft.fft(g.moments()[1][1])[1])
    k = 2 * math.pi / n
    return -math.log(a1 / a0) / (k * k * steps) / (CS2 * (tau - 0.5))


def test_bgk_galilean_defect_against_regularized():
    """The shear stress of BGK carries the cubic-velocity defect the
    third-order regularized equilibrium removes (Sec. II.A): a shear wave
    advected at U = 0.2 decays at a visibly shifted rate under BGK, and at
    the rest rate under the regularized operator."""
    rr = advected_shear_rate("rr", 0.2) - advected_shear_rate("rr", 0.0)
    bgk = advected_shear_rate("bgk", 0.2) - advected_shear_rate("bgk", 0.0)
    assert abs(rr) < 3e-4
    assert abs(bgk) > 3e-2


def test_comparators_refused_where_undefined():
    with pytest.raises(ValueError):
        O.Grid(19, 4, 4, 4, collision="mrt")
    with pytest.raises(ValueError):
        O.Grid(9, 4, 4, 1, collision="bgk", full_order=True)


def test_regularized_more_stable_than_bgk_on_shear_layer():
    """Sec. II.A's stability claim on a D2Q9 64^2 thick shear layer at
    Ma 0.2 over four advection periods: at tau = 0.502 the regularized
    operator stays finite and LBM-BGK diverges."""
    n = 64
    U = 0.2 / math.sqrt(3)
    steps = int(4 * n / U)
    rho, u = W.double_shear_layer(n, U)

    def finite(collision):
        g = O.Grid(9, n, n, 1, tau=0.502, collision=collision).init(rho, u)
        g.step(steps)
        r, uu = g.moments()
        return bool(np.isfinite(r).all() and r.min() > 0 and np.abs(uu).max() < 1)

    assert finite("rr")
    assert not finite("bgk")
