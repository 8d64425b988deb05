"""Pins of the oracle's lattice tables and Hermite basis (Sec. II.A).

The paper cites D2Q9, D3Q19 and D3Q27 as Gauss-Hermite quadratures exact to
second order, and relies on a special property of D2Q9 and D3Q27 to go to
third order.  These tests check the oracle's tables against an independent
tensor-product construction and the quadrature identities, and check which
third-order Hermite polynomials each lattice resolves.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from tests import lattice_ref as R

LATTICES = [9, 19, 27]


@pytest.mark.parametrize("q", LATTICES)
def test_table_matches_independent_construction(q):
    xi, w, opp = O.lattice(q)
    rx, rw = R.lattice(q)
    assert xi.shape == (q, 3)
    got = {tuple(v): wi for v, wi in zip(xi, w)}
    ref = {tuple(v): wi for v, wi in zip(rx, rw)}
    assert set(got) == set(ref)
    for k in ref:
        assert got[k] == pytest.approx(ref[k], abs=1e-16)
    # documented ordering: rest first, then opposite pairs (odd i, i + 1)
    assert tuple(xi[0]) == (0, 0, 0)
    for i in range(1, q, 2):
        assert np.all(xi[i] == -xi[i + 1])
        assert opp[i] == i + 1 and opp[i + 1] == i
    assert opp[0] == 0


@pytest.mark.parametrize("q", LATTICES)
def test_quadrature_isotropy(q):
    xi, w, _ = O.lattice(q)
    d = R.dim(q)
    x = xi[:, :d].astype(float)
    cs2 = 1.0 / 3.0
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, x), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, x, x), cs2 * np.eye(d), atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, x, x, x), 0, atol=1e-16)
    I = np.eye(d)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                       + np.einsum("ad,bc->abcd", I, I))
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, x, x, x, x), iso4, atol=1e-16)


@pytest.mark.parametrize("q", LATTICES)
def test_third_order_basis_orthogonal_with_stated_norms(q):
    """The per-lattice third-order basis is orthogonal (lattice inner product
    sum_i w_i P_i Q_i) to itself and to all lower orders, with norms
    2 cs^6 for xxy-type, cs^6 for xyz, and for the D3Q19 pairs 2 cs^6 (sum)
    and 6 cs^6 (difference)."""
    xi, w = R.lattice(q)
    cs6 = (1.0 / 3.0) ** 3
    basis = R.third_order_basis(q)
    P = np.array([R.basis_poly(xi, c) for _, c in basis])
    G = np.einsum("i,ki,li->kl", w, P, P)
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-15
    norms = np.diag(G)
    for (name, combo), nrm in zip(basis, norms):
        if q == 19:
            expect = 2 * cs6 if list(combo.values()) == [1, 1] else 6 * cs6
        elif name == "xyz":
            expect = cs6
        else:
            expect = 2 * cs6
        assert nrm == pytest.approx(expect, rel=1e-13), name
    d = R.dim(q)
    lower = [np.ones(len(w))] + [xi[:, a].astype(float) for a in range(d)]
    lower += [R.H2(xi, a, b) for a in range(d) for b in range(a, d)]
    for L in lower:
        assert np.abs(np.einsum("i,ki,i->k", w, P, L)).max() < 1e-15


def test_d3q19_does_not_separate_xxy_from_yzz():
    """Sec. II.A: only D2Q9 and D3Q27 have the property that lets the
    expansion go past second order componentwise; on D3Q19 H_xxy and H_yzz
    are not orthogonal (inner product -cs^6) and H_xyz vanishes."""
    xi, w = R.lattice(19)
    g = np.sum(w * R.H3(xi, 0, 0, 1) * R.H3(xi, 1, 2, 2))
    assert g == pytest.approx(-(1.0 / 3.0) ** 3, abs=1e-16)
    assert np.abs(R.H3(xi, 0, 1, 2)).max() == 0.0


def test_splitmix64_published_vector():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")
    want = [int(s) for s in open(path).read().split("\n") if s and not s.startswith("#")]
    got = [O.splitmix64(1234567, k) for k in range(len(want))]
    assert got == want
