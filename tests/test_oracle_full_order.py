"""Pins of the oracle's full recursive regularization (Sec. II.A, expansion
to order n > 2 on D2Q9 and D3Q27) against closed forms:

- the full-order equilibrium of a tensor-product lattice is the product of
  the three-velocity 1D equilibria (all Hermite coefficients rho u..u);
- every Hermite moment of the rebuilt non-equilibrium part equals the
  recursion's coefficient, written out here component by component;
- truncated to third order, the full expansion is the third-order scheme;
- the collision conserves mass and momentum and relaxes the stress.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def he(n, x):
    return np.ones_like(x) if n == 0 else (x if n == 1 else x * x - CS2)


def multi_indices(q):
    d = 2 if q == 9 else 3
    rng = [range(3)] * d + [range(1)] * (3 - d)
    return [k for k in itertools.product(*rng)]


def hermite_moment(q, f, k):
    """sum_i f_i He_kx(xi_x) He_ky(xi_y) He_kz(xi_z)"""
    xi, _, _ = O.lattice(q)
    H = np.ones(q)
    for a in range(3):
        H = H * he(k[a], xi[:, a].astype(float))
    return float(f @ H)


def rand_state(seed, d):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.15, 0.15, 3)
    a2 = rng.normal(0.0, 1e-2, 6)
    if d == 2:
        u[2] = 0.0
        a2[[2, 4, 5]] = 0.0
    return rng.uniform(0.9, 1.1), u, a2


def test_full_equilibrium_is_product_of_1d_equilibria():
    for q in (9, 27):
        d = 2 if q == 9 else 3
        xi, _, _ = O.lattice(q)
        for seed in range(5):
            rho, u, _ = rand_state(seed, d)
            feq = O.equilibrium(q, rho, u, full=True)

            def f1(c, v):  # three-velocity 1D equilibrium, second order
                return (2.0 / 3.0) * (1 - 1.5 * v * v) if c == 0 else (1 + 3 * c * v + 3 * v * v) / 6

            ref = np.array([rho * np.prod([f1(xi[i, a], u[a]) for a in range(d)])
                            for i in range(q)])
            np.testing.assert_allclose(feq, ref, rtol=1e-14, atol=1e-16)


def test_full_equilibrium_moments_are_rho_u_products():
    for q in (9, 27):
        d = 2 if q == 9 else 3
        rho, u, _ = rand_state(11, d)
        feq = O.equilibrium(q, rho, u, full=True)
        for k in multi_indices(q):
            want = rho * u[0] ** k[0] * u[1] ** k[1] * u[2] ** k[2]
            assert hermite_moment(q, feq, k) == pytest.approx(want, abs=1e-15)


def neq_closed_forms(u, a2):
    """Recursion coefficients written out for the components pinned here
    (a2 packed xx, yy, zz, xy, xz, yz)."""
    ux, uy, uz = u
    xx, yy, zz, xy, xz, yz = a2
    return {
        (2, 0, 0): xx, (0, 2, 0): yy, (1, 1, 0): xy, (1, 0, 1): xz, (0, 1, 1): yz,
        (2, 1, 0): uy * xx + 2 * ux * xy,
        (1, 2, 0): ux * yy + 2 * uy * xy,
        (1, 1, 1): ux * yz + uy * xz + uz * xy,
        (2, 2, 0): uy * uy * xx + ux * ux * yy + 4 * ux * uy * xy,
        (2, 1, 1): uy * uz * xx + 2 * ux * uz * xy + 2 * ux * uy * xz + ux * ux * yz,
        (2, 2, 1): (uy * uy * uz * xx + ux * ux * uz * yy + 4 * ux * uy * uz * xy
                    + 2 * ux * uy * uy * xz + 2 * ux * ux * uy * yz),
        (2, 2, 2): (uy * uy * uz * uz * xx + ux * ux * uz * uz * yy + ux * ux * uy * uy * zz
                    + 4 * ux * uy * uz * uz * xy + 4 * ux * uz * uy * uy * xz
                    + 4 * uy * uz * ux * ux * yz),
    }


@pytest.mark.parametrize("q", [9, 27])
def test_full_noneq_moments_follow_the_recursion(q):
    d = 2 if q == 9 else 3
    for seed in range(4):
        _, u, a2 = rand_state(20 + seed, d)
        fneq = O.noneq(q, u, a2, full=True)
        forms = neq_closed_forms(u, a2)
        for k in multi_indices(q):
            m = hermite_moment(q, fneq, k)
            if sum(k) < 2:
                assert abs(m) < 1e-16
            elif k in forms:
                assert m == pytest.approx(forms[k], rel=1e-12, abs=1e-17), k


@pytest.mark.parametrize("q", [9, 27])
def test_third_order_truncation_of_full_expansion(q):
    """Both expansions carry the same moments up to third order; the full
    one adds fourth and higher."""
    d = 2 if q == 9 else 3
    rho, u, a2 = rand_state(31, d)
    for full_f, third_f in ((O.equilibrium(q, rho, u, full=True), O.equilibrium(q, rho, u)),
                            (O.noneq(q, u, a2, full=True), O.noneq(q, u, a2))):
        high = 0.0
        for k in multi_indices(q):
            a, b = hermite_moment(q, full_f, k), hermite_moment(q, third_f, k)
            if sum(k) <= 3:
                assert a == pytest.approx(b, abs=1e-15)
            else:
                assert abs(b) < 1e-15
                high = max(high, abs(a))
        assert high > 1e-6


@pytest.mark.parametrize("q", [9, 27])
@pytest.mark.parametrize("chi", [0.0, 0.3])
def test_full_collision_moments(q, chi):
    d = 2 if q == 9 else 3
    rng = np.random.default_rng(40)
    rho, u, a2 = rand_state(41, d)
    f = O.equilibrium(q, rho, u) + O.noneq(q, u, a2) + 1e-4 * rng.normal(size=q)
    xi, _, _ = O.lattice(q)
    tau, rho_ref, u_ref = 0.7, 1.02, np.array([0.05, -0.02, 0.01 if d == 3 else 0.0])
    post = O.collide(q, f, tau, chi=chi, rho_ref=rho_ref, u_ref=u_ref, full=True)
    r, j = f.sum(), f @ xi
    rs = (r + 0.5 * chi * rho_ref) / (1 + 0.5 * chi)
    js = (j + 0.5 * chi * rho_ref * u_ref) / (1 + 0.5 * chi)
    assert post.sum() == pytest.approx((1 - chi) * rs + chi * rho_ref, rel=1e-14)
    np.testing.assert_allclose(post @ xi, (1 - chi) * js + chi * rho_ref * u_ref,
                               rtol=1e-12, atol=1e-16)
    if chi == 0.0:
        us = js / rs
        Pi = (f[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0)
        a2n = Pi - rs * CS2 * np.eye(3) - rs * np.outer(us, us)
        Pp = (post[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0)
        want = rs * CS2 * np.eye(3) + rs * np.outer(us, us) + (1 - 1 / tau) * a2n
        np.testing.assert_allclose(Pp[:d, :d], want[:d, :d], rtol=1e-12, atol=1e-15)


def test_full_order_refused_on_d3q19():
    with pytest.raises(ValueError):
        O.equilibrium(19, 1.0, (0.1, 0, 0), full=True)
    with pytest.raises(ValueError):
        O.Grid(19, 4, 4, 4, full_order=True)


def test_full_order_grid_viscosity_and_conservation():
    """Shear-wave decay on D2Q9 at the full order gives nu = cs^2 (tau - 1/2)
    as the third-order scheme does, advected or not; mass and momentum stay
    constant to rounding."""
    n, tau, A = 64, 0.6, 1e-3
    nu = CS2 * (tau - 0.5)
    k = 2 * math.pi / n
    y = np.repeat(np.arange(n), n).astype(float)
    for U in (0.0, 0.15):
        u = np.zeros((3, n * n))
        u[0] = U + A * np.sin(k * y)
        g = O.Grid(9, n, n, 1, tau=tau, full_order=True).init(np.ones(n * n), u)
        m0, j0 = g.f.sum(), g.moments()[1][0].sum()
        steps = 400
        g.step(steps)
        r, uu = g.moments()
        amp = 2 * (uu[0] - uu[0].mean()) @ np.sin(k * y) / (n * n)
        # an advected wave moves along x only, the y-profile stays a sine
        rate = -math.log(abs(amp) / A) / steps
        assert rate == pytest.approx(nu * k * k, rel=2e-2)
        assert abs(g.f.sum() - m0) < 1e-11 * m0
        assert abs(uu[0].sum() - j0) < 1e-9 * max(abs(j0), 1.0) + 1e-12
