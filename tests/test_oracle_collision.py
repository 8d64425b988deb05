"""Pins of the oracle's one-cell collision (Sec. II.A and II.C).

Each check is a property the paper states or the mathematics fixes, chosen so
that a dropped term, a wrong sign or index, or a wrong norm in the oracle
fails at least one of them.
"""
import numpy as np
import pytest

import oracle as O
from tests import lattice_ref as R

LATTICES = [9, 19, 27]
CS2 = 1.0 / 3.0


def rand_state(q, rng, amp_u=0.1, amp_a2=2e-3):
    d = R.dim(q)
    rho = rng.uniform(0.9, 1.1)
    u = np.zeros(3)
    u[:d] = rng.uniform(-amp_u, amp_u, d)
    a2 = np.zeros(6)
    a2[[0, 1, 3]] = rng.uniform(-amp_a2, amp_a2, 3)
    if d == 3:
        a2[[2, 4, 5]] = rng.uniform(-amp_a2, amp_a2, 3)
    return rho, u, a2


def full2(a2):
    return np.array([[a2[0], a2[3], a2[4]], [a2[3], a2[1], a2[5]], [a2[4], a2[5], a2[2]]])


def recursion_a3(u, a2):
    """eq. (recursive2) at n = 3 for the non-equilibrium coefficient."""
    A = full2(a2)
    return (np.einsum("a,bc->abc", u, A) + np.einsum("b,ac->abc", u, A)
            + np.einsum("c,ab->abc", u, A))


@pytest.mark.parametrize("q", LATTICES)
def test_rebuild_reproduces_rho_j_pi(q):
    """The rebuilt populations carry exactly rho, rho u and
    Pi = rho cs^2 I + rho u u + a2_neq (eqs. Hcoeff, HEeqAndNeq)."""
    rng = np.random.default_rng(q)
    xi, _, _ = O.lattice(q)
    d = R.dim(q)
    for _ in range(20):
        rho, u, a2 = rand_state(q, rng)
        f = O.equilibrium(q, rho, u) + O.noneq(q, u, a2)
        r, j, Pi, _ = R.moments(xi, f)
        assert r == pytest.approx(rho, abs=1e-15)
        np.testing.assert_allclose(j, rho * u, atol=1e-15)
        want = rho * CS2 * np.eye(3) + rho * np.outer(u, u) + full2(a2)
        np.testing.assert_allclose(Pi[:d, :d], want[:d, :d], atol=1e-15)
        # the non-equilibrium part alone carries no mass or momentum
        fn = O.noneq(q, u, a2)
        r2, j2, _, _ = R.moments(xi, fn)
        assert abs(r2) < 1e-16 and np.abs(j2).max() < 1e-16


@pytest.mark.parametrize("q", LATTICES)
def test_third_order_targets_in_supported_basis(q):
    """In every third-order direction the lattice resolves, the equilibrium
    carries rho u u u (eq. recursive1) and the non-equilibrium part carries
    the recursive coefficient of eq. (recursive2)."""
    rng = np.random.default_rng(100 + q)
    xi, w, _ = O.lattice(q)
    basis = R.third_order_basis(q)
    for _ in range(20):
        rho, u, a2 = rand_state(q, rng)
        feq = O.equilibrium(q, rho, u)
        fne = O.noneq(q, u, a2)
        a3eq = rho * np.einsum("a,b,c->abc", u, u, u)
        a3ne = recursion_a3(u, a2)
        for name, combo in basis:
            P = R.basis_poly(xi, combo)
            assert np.dot(feq, P) == pytest.approx(R.basis_target(a3eq, combo), abs=1e-16), name
            assert np.dot(fne, P) == pytest.approx(R.basis_target(a3ne, combo), abs=1e-16), name


@pytest.mark.parametrize("q", LATTICES)
def test_offdiagonal_third_moment_exact_diagonal_aliased(q):
    """Sec. II.A: with the extended equilibrium the off-diagonal third moments
    are exact, sum f_eq xi_x^2 xi_y = rho (u_x^2 u_y + cs^2 u_y), while the
    diagonal ones stay aliased (xi^3 = xi on the lattice)."""
    rng = np.random.default_rng(200 + q)
    xi, _, _ = O.lattice(q)
    d = R.dim(q)
    for _ in range(10):
        rho, u, _ = rand_state(q, rng, amp_u=0.2)
        f = O.equilibrium(q, rho, u)
        _, _, _, Q = R.moments(xi, f)
        for a in range(d):
            for b in range(d):
                if a != b:
                    want = rho * (u[a] ** 2 * u[b] + CS2 * u[b])
                    assert Q[a, a, b] == pytest.approx(want, abs=1e-16)
            assert Q[a, a, a] == pytest.approx(rho * u[a], abs=1e-16)


@pytest.mark.parametrize("q", LATTICES)
def test_equilibrium_is_fixed_point(q):
    rng = np.random.default_rng(300 + q)
    for _ in range(20):
        rho, u, _ = rand_state(q, rng, amp_u=0.2)
        feq = O.equilibrium(q, rho, u)
        tau = rng.uniform(0.51, 2.0)
        np.testing.assert_allclose(O.collide(q, feq, tau), feq, atol=2e-16)


@pytest.mark.parametrize("q", LATTICES)
def test_collision_conserves_and_relaxes_stress(q):
    """Mass and momentum are conserved; the non-equilibrium stress leaves the
    collision multiplied by (1 - 1/tau) (eq. optimizedLB)."""
    rng = np.random.default_rng(400 + q)
    xi, _, _ = O.lattice(q)
    d = R.dim(q)
    for _ in range(20):
        f = O.equilibrium(q, *rand_state(q, rng)[:2]) + rng.uniform(-1e-3, 1e-3, q)
        tau = rng.uniform(0.51, 2.0)
        post = O.collide(q, f, tau)
        r0, j0, Pi0, _ = R.moments(xi, f)
        r1, j1, Pi1, _ = R.moments(xi, post)
        assert r1 == pytest.approx(r0, abs=1e-15)
        np.testing.assert_allclose(j1, j0, atol=1e-15)
        u = j0 / r0
        Peq = r0 * CS2 * np.eye(3) + r0 * np.outer(u, u)
        np.testing.assert_allclose((Pi1 - Peq)[:d, :d], (1 - 1 / tau) * (Pi0 - Peq)[:d, :d],
                                   atol=1e-15)


@pytest.mark.parametrize("q", LATTICES)
def test_regularization_discards_higher_order_content(q):
    """Sec. II.A (Latt-Chopard procedure): the post-collision state depends
    only on rho, u and a2_neq, so adding any population vector with zero
    moments up to second order changes nothing."""
    rng = np.random.default_rng(500 + q)
    xi, _, _ = O.lattice(q)
    d = R.dim(q)
    x = xi[:, :d].astype(float)
    rows = [np.ones(q)] + [x[:, a] for a in range(d)]
    rows += [x[:, a] * x[:, b] for a in range(d) for b in range(a, d)]
    M = np.array(rows)
    _, _, vt = np.linalg.svd(M)
    null = vt[len(rows):]
    assert null.shape[0] == q - len(rows)
    for _ in range(10):
        rho, u, a2 = rand_state(q, rng)
        f = O.equilibrium(q, rho, u) + O.noneq(q, u, a2)
        g = null.T @ rng.uniform(-1e-3, 1e-3, null.shape[0])
        np.testing.assert_allclose(O.collide(q, f + g, 0.7), O.collide(q, f, 0.7), atol=1e-16)


@pytest.mark.parametrize("q", LATTICES)
def test_sponge_reference_state_is_fixed_point(q):
    """eq. (dampingLBM): the force vanishes at the reference state."""
    rng = np.random.default_rng(600 + q)
    for _ in range(10):
        rho, u, _ = rand_state(q, rng)
        feq = O.equilibrium(q, rho, u)
        chi = rng.uniform(0, 1.5)
        np.testing.assert_allclose(O.collide(q, feq, 0.8, chi, rho, u), feq, atol=2e-16)


@pytest.mark.parametrize("q", LATTICES)
def test_sponge_chi_zero_is_rrbgk(q):
    """Sec. II.C: with chi = 0 the damped update is eq. (optimizedLB)."""
    rng = np.random.default_rng(650 + q)
    rho, u, a2 = rand_state(q, rng)
    f = O.equilibrium(q, rho, u) + O.noneq(q, u, a2) + rng.uniform(-1e-4, 1e-4, q)
    np.testing.assert_array_equal(O.collide(q, f, 0.7, 0.0, 1.3, (0.1, 0.1, 0.1)),
                                  O.collide(q, f, 0.7))


def homogeneous_decay(collide, q, tau, chi, delta=1e-2):
    """One collision of a uniform state rho = 1 + delta at rest with the
    sponge reference (1, 0): return the factor g on the density deviation."""
    f = O.equilibrium(q, 1.0 + delta, (0, 0, 0))
    post = collide(q, f, tau, chi, 1.0, (0, 0, 0))
    return (post.sum() - 1.0) / delta


@pytest.mark.parametrize("q", LATTICES)
def test_sponge_bgk_decay_matches_printed_sigma_eff(q):
    """eq. (effectiveCoefficient): with the modified moments of
    eq. (modifiedMoments) at n = m = 1/2 and the force added in full, the
    homogeneous BGK density mode decays per step by g, and its trapezoidal
    rate 2(1-g)/(1+g) equals sigma_eff = (1 + 1/(2 tau)) chi / (1 - chi/(4 tau))."""
    for tau in (0.51, 0.6, 0.8, 1.0, 1.7):
        for chi in (0.01, 0.1, 0.3, 0.9, 1.9):
            if chi >= 4 * tau:
                continue
            g = homogeneous_decay(O.collide_bgk, q, tau, chi)
            rate = 2 * (1 - g) / (1 + g)
            sigma_eff = (1 + 1 / (2 * tau)) * chi / (1 - chi / (4 * tau))
            assert rate == pytest.approx(sigma_eff, rel=1e-9)
            # stability bound chi < 4 tau  <=>  1 + g > 0
            assert 1 + g > 0


@pytest.mark.parametrize("q", LATTICES)
def test_sponge_regularized_decay(q):
    """The regularized f_neq carries no mass, so the damped density mode of
    the regularized operator decays by g = (1 - chi)/(1 + chi/2) whatever tau
    is; its trapezoidal rate is the printed sigma_eff at tau = 1."""
    for chi in (0.01, 0.2, 0.5, 1.2):
        for tau in (0.52, 0.9):
            g = homogeneous_decay(O.collide, q, tau, chi)
            assert g == pytest.approx((1 - chi) / (1 + chi / 2), rel=1e-9)
        rate = 2 * (1 - g) / (1 + g)
        assert rate == pytest.approx((1 + 0.5) * chi / (1 - chi / 4), rel=1e-9)


def test_sponge_profile_closed_form():
    """Sec. II.C polynomial profile: zero at the inner edge, maximum 1 at
    four fifths of the width, mirrored on the low face; faces combine by max."""
    nx, W, chi_max = 100, 20, 0.25
    g = O.Grid(9, nx, 8, 1, sponge_width=(W, W, 0, 0, 0, 0), chi_max=chi_max)
    s0, L = nx - W, nx
    for x in range(nx):
        s = x if x >= s0 else nx - 1 - x
        want = 0.0
        if s >= s0:
            want = chi_max * 3125 * (L - s) * (s - s0) ** 4 / (256 * (L - s0) ** 5)
        assert g.chi(x, 3) == pytest.approx(want, abs=1e-15)
    assert g.chi(s0 + 16, 0) == pytest.approx(chi_max, abs=1e-15)
    assert g.chi(nx - 1 - (s0 + 16), 0) == pytest.approx(chi_max, abs=1e-15)
    assert g.chi(s0, 0) == 0.0 and g.chi(nx // 2, 0) == 0.0
    g2 = O.Grid(9, 40, 40, 1, sponge_width=(0, 10, 0, 10, 0, 0), chi_max=1.0)
    assert g2.chi(38, 32) == pytest.approx(max(g2.chi(38, 0), g2.chi(0, 32)), abs=1e-15)
