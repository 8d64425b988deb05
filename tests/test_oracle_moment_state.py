"""Pins of the moment-stored state on the oracle (CPU): without an absorbing
layer the regularized collision leaves every cell exactly at
E(rho, u) + N(a2*, u) with a2* = Pi* - rho cs^2 I - rho u u the
post-collision non-equilibrium stress (eqs. eqH, neqH, recursive1,
recursive2: every Hermite coefficient follows from rho, u and a2_neq, and
the non-equilibrium part is linear in a2_neq).  Ten numbers per cell
therefore carry the whole state; with a sponge, or with the BGK comparator,
the post-collision state leaves that span, which is why the moment storages
refuse both.
"""
import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def post_moments(q, f):
    xi, _, _ = O.lattice(q)
    rho = f.sum()
    j = (f[:, None] * xi).sum(axis=0)
    u = j / rho
    Pi = np.einsum("i,ia,ib->ab", f, xi, xi)
    a2 = Pi - rho * CS2 * np.eye(3) - rho * np.outer(u, u)
    packed = np.array([a2[0, 0], a2[1, 1], a2[2, 2], a2[0, 1], a2[0, 2], a2[1, 2]])
    return rho, u, packed


def generic_cell(q, rng):
    """Pre-collision populations with content at every order: an
    equilibrium plus a random perturbation (rest mass kept positive)."""
    u = rng.uniform(-0.08, 0.08, 3)
    if q == 9:
        u[2] = 0.0
    f = O.equilibrium(q, 1.0 + rng.uniform(-0.02, 0.02), u)
    _, w, _ = O.lattice(q)
    return f + 1e-3 * w * rng.standard_normal(q)


@pytest.mark.parametrize("q,full", [(9, False), (19, False), (27, False), (9, True),
                                    (27, True)])
@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 1.7])
def test_regularized_post_state_is_its_moment_rebuild(q, full, tau):
    rng = np.random.default_rng(q * 100 + int(tau * 10) + full)
    for _ in range(20):
        f = generic_cell(q, rng)
        post = O.collide(q, f, tau, full=full)
        rho, u, a2 = post_moments(q, post)
        rebuilt = O.equilibrium(q, rho, u, full=full) + O.noneq(q, u, a2, full=full)
        assert np.max(np.abs(rebuilt - post)) <= 1e-14 * np.max(np.abs(post))


@pytest.mark.parametrize("q", [9, 19, 27])
def test_absorbing_layer_and_bgk_leave_the_span(q):
    """The damping force mixes two equilibria, whose third-order content is
    not the recursion of the mixed stress; BGK keeps the pre-collision
    higher-order content.  Either state differs from its moment rebuild."""
    rng = np.random.default_rng(7 + q)
    f = generic_cell(q, rng)
    u_ref = (0.1, -0.05, 0.02) if q != 9 else (0.1, -0.05, 0.0)
    for post in (O.collide(q, f, 0.6, chi=0.3, rho_ref=1.01, u_ref=u_ref),
                 O.collide_bgk(q, f, 0.6)):
        rho, u, a2 = post_moments(q, post)
        rebuilt = O.equilibrium(q, rho, u) + O.noneq(q, u, a2)
        assert np.max(np.abs(rebuilt - post)) > 1e-7 * np.max(np.abs(post))
