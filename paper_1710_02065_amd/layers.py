"""Absorbing-layer fields for lbm_set_sponge (Sec. II.C with the layer
geometries and references of Sec. III and IV): host-side builders of chi,
rho_ref and u_ref over a grid's cells (FP64 numpy arrays, cell index
c = (z ny + y) nx + x).

- face_layer: the planar layers of the faces as a field (to pair with a
  spatially varying reference);
- circular_layer: the layer of the cylinder setup, a ring (2D) or shell
  (3D) whose strength follows the profile of Sec. II.C in the distance from
  a centre;
- jet_reference: a round free jet's self-similar mean velocity as the
  reference the outflow layers relax to (the jet setup of Sec. IV), in place
  of a constant.
"""
import math

import numpy as np


def profile(s, s0, L):
    """Sec. II.C profile 3125 (L - s)(s - s0)^4 / (256 (L - s0)^5) on
    [s0, L], zero outside; its maximum 1 is at s0 + 4/5 (L - s0)."""
    s = np.asarray(s, dtype=np.float64)
    d = np.clip((s - s0) / (L - s0), 0.0, 1.0)
    return (3125.0 / 256.0) * (1.0 - d) * d ** 4


def _coords(shape):
    nx, ny, nz = shape
    c = np.arange(nx * ny * nz)
    return (c % nx).astype(np.float64), ((c // nx) % ny).astype(np.float64), \
        (c // (nx * ny)).astype(np.float64)


def face_layer(shape, widths, chi_max):
    """chi per cell of the planar face layers (the profile the sweep
    evaluates from the coordinates when no field is given): on face f
    (x-, x+, y-, y+, z-, z+) of width W the profile over the last W cells,
    s = distance coordinate from the opposite side, s0 = n - W, L = n;
    faces combine by their maximum."""
    pos = _coords(shape)
    chi = np.zeros(pos[0].size)
    for f, W in enumerate(widths):
        if W <= 0:
            continue
        ax, n = f // 2, shape[f // 2]
        s = pos[ax] if f % 2 == 1 else (n - 1) - pos[ax]
        chi = np.maximum(chi, profile(s, float(n - W), float(n)))
    return chi_max * chi


def circular_layer(shape, center, r0, r1, chi_max):
    """chi per cell: chi_max times the profile in the distance r from
    `center` between r0 (inner edge) and r1; use r1 at least the largest
    distance in the grid so that the outermost cells stay absorbing."""
    x, y, z = _coords(shape)
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2
    if shape[2] > 1:
        r2 = r2 + (z - center[2]) ** 2
    return chi_max * profile(np.sqrt(r2), r0, r1)


def jet_reference(shape, D, U, inlet=(0.0, None, None), axis=0, x0=-3.0, B=5.8,
                  S=0.094, core=5.0, rho_ref=1.0):
    """Reference (rho_ref [N], u_ref [3][N]) of a round jet of diameter D
    (cells) and exit velocity U issuing along `axis` from the inlet plane
    through the centre of the cross-section (inlet = (plane position,
    centre coordinates or None for the middle)).  Beyond the potential core
    (`core` diameters) the axial velocity is the self-similar far field
    U_c = B U D / (s - x0 D) times (1 + a eta^2)^-2, eta = r / (s - x0 D),
    a = (sqrt 2 - 1) / S^2 (half-width r_1/2 = S (s - x0 D)); inside the
    core, U within r < D/2.  Radial velocity is left at zero."""
    pos = _coords(shape)
    n = shape
    axes = [a for a in range(3) if a != axis and n[a] > 1]
    s = pos[axis] - inlet[0]
    r2 = np.zeros_like(s)
    for k, a in enumerate(axes):
        c = inlet[1 + k] if len(inlet) > 1 + k and inlet[1 + k] is not None else (n[a] - 1) / 2.0
        r2 += (pos[a] - c) ** 2
    r = np.sqrt(r2)
    xe = np.maximum(s - x0 * D, 1e-9)
    a = (math.sqrt(2.0) - 1.0) / (S * S)
    far = np.minimum(B * U * D / xe, U) / (1.0 + a * (r / xe) ** 2) ** 2
    near = np.where(r < 0.5 * D, U, 0.0)
    ua = np.where(s < core * D, near, far)
    u = np.zeros((3, ua.size))
    u[axis] = ua
    return np.full(ua.size, rho_ref), u
