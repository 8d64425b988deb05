"""Test-side lattice constructions, written independently of the oracle.

D2Q9 and D3Q27 are built as tensor products of the D1Q3 Gauss-Hermite rule
(nodes -1, 0, 1 with weights 1/6, 2/3, 1/6); D3Q19 keeps the D3Q27 nodes with
|xi|^2 <= 2 and takes the textbook weights.  Hermite polynomials are written
from their definition (H^n = (-1)^n w^-1 grad^n w for the Gaussian weight in
lattice units, cs^2 = 1/3).
"""
import itertools

import numpy as np

CS2 = 1.0 / 3.0
D1Q3 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}


def tensor_lattice(d):
    xs, ws = [], []
    for t in itertools.product((-1, 0, 1), repeat=d):
        xs.append(list(t) + [0] * (3 - d))
        ws.append(np.prod([D1Q3[c] for c in t]))
    return np.array(xs, dtype=np.int64), np.array(ws)


def lattice(q):
    if q == 9:
        return tensor_lattice(2)
    if q == 27:
        return tensor_lattice(3)
    if q == 19:
        xs, _ = tensor_lattice(3)
        keep = (xs ** 2).sum(1) <= 2
        xs = xs[keep]
        n2 = (xs ** 2).sum(1)
        ws = np.where(n2 == 0, 1.0 / 3, np.where(n2 == 1, 1.0 / 18, 1.0 / 36))
        return xs, ws
    raise ValueError(q)


def dim(q):
    return 2 if q == 9 else 3


def H2(xi, a, b):
    return xi[:, a] * xi[:, b] - CS2 * (a == b)


def H3(xi, a, b, c):
    xa, xb, xc = xi[:, a], xi[:, b], xi[:, c]
    return xa * xb * xc - CS2 * (xa * (b == c) + xb * (a == c) + xc * (a == b))


X, Y, Z = 0, 1, 2


def third_order_basis(q):
    """List of (name, weights over third-order tensor components) that the
    lattice resolves.  Each entry: dict {(a,b,c): coefficient}; the basis
    polynomial is sum coef * H_abc and its target moment sum coef * a_abc."""
    if q == 9:
        return [("xxy", {(X, X, Y): 1}), ("xyy", {(X, Y, Y): 1})]
    if q == 27:
        names = {"xxy": (X, X, Y), "xyy": (X, Y, Y), "xxz": (X, X, Z),
                 "xzz": (X, Z, Z), "yyz": (Y, Y, Z), "yzz": (Y, Z, Z),
                 "xyz": (X, Y, Z)}
        return [(k, {v: 1}) for k, v in names.items()]
    if q == 19:
        out = []
        pairs = [((X, X, Y), (Y, Z, Z)), ((X, Y, Y), (X, Z, Z)), ((X, X, Z), (Y, Y, Z))]
        for p, r in pairs:
            out.append(("+".join(map(str, (p, r))), {p: 1, r: 1}))
            out.append(("-".join(map(str, (p, r))), {p: 1, r: -1}))
        return out
    raise ValueError(q)


def basis_poly(xi, combo):
    return sum(c * H3(xi, *k) for k, c in combo.items())


def basis_target(a3, combo):
    return sum(c * a3[k] for k, c in combo.items())


def moments(xi, f):
    """rho, j[3], Pi[3,3], and the full third moment tensor of populations f."""
    xf = xi.astype(np.float64)
    rho = f.sum()
    j = (f[:, None] * xf).sum(0)
    Pi = np.einsum("i,ia,ib->ab", f, xf, xf)
    Q = np.einsum("i,ia,ib,ic->abc", f, xf, xf, xf)
    return rho, j, Pi, Q
