"""Seeded synthetic inputs: macroscopic initial fields, masks, probe sets and
job streams with the shapes, sizes and structure of the paper's workloads.

This module holds no lattice Boltzmann arithmetic.  It produces plain fields
(density, velocity, strain rate), geometry masks and random draws; the GPU
library and the CPU oracle each turn them into populations with their own
code.  Every random draw is numpy's PCG64 seeded from the arguments.

Field layout: flat arrays over cells with x fastest, index (z*ny + y)*nx + x;
vector fields are [3][N] (z component zero in 2D); strain-rate fields are
[6][N] in the order (xx, yy, zz, xy, xz, yz).

The paper's applications (a cylinder in uniform flow, Sec. III; a round jet,
Sec. IV) need comparison datasets and multi-level setups that are not
reproduced here; the generators below are synthetic stand-ins with the same
Mach and Reynolds numbers and geometry proportions.
"""
import math

import numpy as np

CS2 = 1.0 / 3.0
CS = math.sqrt(CS2)

FLUID, SOLID, INLET = 0, 1, 2


def _grid(nx, ny, nz=1):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel().astype(np.float64), y.ravel().astype(np.float64), z.ravel().astype(np.float64)


def taylor_green_2d(n, U, rho0=1.0):
    """Decaying 2D Taylor-Green vortex on an n x n periodic box:
    u_x = -U cos kx sin ky, u_y = U sin kx cos ky, k = 2 pi / n, with the
    matching incompressible pressure turned into density through p = cs^2 rho.
    Returns rho [N], u [3][N], strain rate S [6][N]."""
    x, y, _ = _grid(n, n)
    k = 2 * math.pi / n
    N = n * n
    u = np.zeros((3, N))
    u[0] = -U * np.cos(k * x) * np.sin(k * y)
    u[1] = U * np.sin(k * x) * np.cos(k * y)
    rho = rho0 - rho0 * U * U / (4 * CS2) * (np.cos(2 * k * x) + np.cos(2 * k * y))
    S = np.zeros((6, N))
    S[0] = U * k * np.sin(k * x) * np.sin(k * y)
    S[1] = -S[0]
    # S_xy = (du_x/dy + du_y/dx) / 2 vanishes for this vortex
    return rho, u, S


def taylor_green_mode_2d(n):
    """The x-velocity shape -cos kx sin ky of the 2D Taylor-Green vortex."""
    x, y, _ = _grid(n, n)
    k = 2 * math.pi / n
    return -np.cos(k * x) * np.sin(k * y)


def taylor_green_3d(n, U, rho0=1.0, pulse_amp=0.0, pulse_sigma=8.0, center=None):
    """3D Taylor-Green vortex on an n^3 periodic box,
    u = U (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0), with its
    incompressible pressure p - p0 = rho0 U^2/16 (cos 2kx + cos 2ky)(cos 2kz + 2)
    as a density perturbation, plus an optional Gaussian acoustic pulse of
    relative amplitude pulse_amp and width pulse_sigma at `center`."""
    x, y, z = _grid(n, n, n)
    k = 2 * math.pi / n
    N = n ** 3
    u = np.zeros((3, N))
    u[0] = U * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    u[1] = -U * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    dp = rho0 * U * U / 16.0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (np.cos(2 * k * z) + 2.0)
    rho = rho0 + dp / CS2
    if pulse_amp:
        c = (n / 2.0,) * 3 if center is None else center
        r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
        rho = rho + pulse_amp * rho0 * np.exp(-r2 / (2 * pulse_sigma ** 2))
    return rho, u


def plane_pulse(nx, ny, nz=1, amp=1e-4, sigma=8.0, x0=None, rho0=1.0):
    """Plane Gaussian density pulse along x at rest (acoustic test)."""
    x, _, _ = _grid(nx, ny, nz)
    x0 = nx / 2.0 if x0 is None else x0
    rho = rho0 * (1.0 + amp * np.exp(-((x - x0) ** 2) / (2 * sigma ** 2)))
    return rho, np.zeros((3, nx * ny * nz))


def double_shear_layer(n, U, width=80.0, delta=0.05):
    """Doubly periodic thick shear layer on an n x n box (Brown & Minion
    1995): u_x = U tanh(width (y/n - 1/4)) below the middle and
    U tanh(width (3/4 - y/n)) above, u_y = delta U sin(2 pi (x/n + 1/4)),
    uniform density.  Returns rho [N], u [3][N]."""
    x, y, _ = _grid(n, n)
    yn, xn = y / n, x / n
    u = np.zeros((3, n * n))
    u[0] = np.where(yn <= 0.5, U * np.tanh(width * (yn - 0.25)),
                    U * np.tanh(width * (0.75 - yn)))
    u[1] = delta * U * np.sin(2 * math.pi * (xn + 0.25))
    return np.ones(n * n), u


def shear_wave(nx, ny, nz, amp, k_axis=0, u_axis=1, advect=(0.0, 0.0, 0.0), mode=1):
    """Sinusoidal shear wave u_{u_axis} = amp sin(2 pi mode s / n_s) varying
    along k_axis, on top of a uniform velocity `advect`."""
    pos = _grid(nx, ny, nz)
    n = (nx, ny, nz)[k_axis]
    k = 2 * math.pi * mode / n
    N = nx * ny * nz
    u = np.zeros((3, N))
    for a in range(3):
        u[a] += advect[a]
    u[u_axis] += amp * np.sin(k * pos[k_axis])
    return np.ones(N), u


def random_state(shape, seed, d, u_amp=0.05, rho_amp=0.02, pi_amp=1e-3, rho0=1.0):
    """Random (white) density, velocity and non-equilibrium stress fields for
    single-step parity checks from generic states."""
    nx, ny, nz = shape
    N = nx * ny * nz
    rng = np.random.default_rng(seed)
    rho = rho0 * (1.0 + rng.uniform(-rho_amp, rho_amp, N))
    u = np.zeros((3, N))
    u[:d] = rng.uniform(-u_amp, u_amp, (d, N))
    p = np.zeros((6, N))
    comps = [0, 1, 3] if d == 2 else [0, 1, 2, 3, 4, 5]
    p[comps] = rng.uniform(-pi_amp, pi_amp, (len(comps), N))
    return rho, u, p


def uniform_perturbed(shape, U, u_dir, seed, rel_noise, d, rho0=1.0):
    """Uniform flow U * u_dir with a seeded relative velocity perturbation
    (uniform in [-1, 1) times rel_noise * U per component)."""
    nx, ny, nz = shape
    N = nx * ny * nz
    rng = np.random.default_rng(seed)
    u = np.zeros((3, N))
    for a in range(d):
        u[a] = U * u_dir[a]
    u[:d] += rel_noise * U * rng.uniform(-1.0, 1.0, (d, N))
    return np.full(N, rho0), u


def cylinder_mask(nx, ny, D, cx, cy, inlet_column=True):
    """SOLID disc of diameter D centred at (cx, cy) (cell centres inside the
    circle), plus an INLET column at x = 0."""
    x, y, _ = _grid(nx, ny)
    m = np.zeros(nx * ny, dtype=np.uint8)
    m[(x - cx) ** 2 + (y - cy) ** 2 <= (D / 2.0) ** 2] = SOLID
    if inlet_column:
        m[x == 0] = INLET
    return m


def cylinder_probes(nx, ny, D, cx, cy, radii=(1.5, 2.0, 3.0, 4.0), angles_deg=(90.0, 78.2)):
    """Probe cells at r = radii * D along the given angles from the flow
    direction (angle 90 = straight up from the cylinder centre)."""
    cells = []
    for ang in angles_deg:
        a = math.radians(ang)
        for r in radii:
            px = int(round(cx + r * D * math.cos(a)))
            py = int(round(cy + r * D * math.sin(a)))
            px = min(max(px, 0), nx - 1)
            py = min(max(py, 0), ny - 1)
            cells.append(py * nx + px)
    return np.array(cells, dtype=np.int64)


def closed_box_mask(nx, ny, nz=1):
    """Fluid box enclosed by one layer of SOLID cells on every face."""
    x, y, z = _grid(nx, ny, nz)
    m = np.zeros(nx * ny * nz, dtype=np.uint8)
    wall = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1)
    if nz > 1:
        wall |= (z == 0) | (z == nz - 1)
    m[wall] = SOLID
    return m


def channel_walls_mask(nx, ny, nz=1, axis=1):
    """SOLID rows at both ends of `axis` (a plane channel)."""
    pos = _grid(nx, ny, nz)
    n = (nx, ny, nz)[axis]
    m = np.zeros(nx * ny * nz, dtype=np.uint8)
    m[(pos[axis] == 0) | (pos[axis] == n - 1)] = SOLID
    return m


def jet_inlet_mask(nx, ny, nz, D):
    """INLET disc of diameter D (cell centres inside) at the centre of the
    x = 0 face; the rest of the face is left FLUID (zero-gradient outflow)."""
    x, y, z = _grid(nx, ny, nz)
    cy, cz = (ny - 1) / 2.0, (nz - 1) / 2.0
    m = np.zeros(nx * ny * nz, dtype=np.uint8)
    m[(x == 0) & ((y - cy) ** 2 + (z - cz) ** 2 <= (D / 2.0) ** 2)] = INLET
    return m


def serving_jobs(n_jobs, seed, rate_per_s, side_range=(256, 2048), ma_range=(0.05, 0.3),
                 step_range=(2000, 20000), step_scale=1.0):
    """Poisson stream of 2D serving jobs: arrival times (s), kind
    ('cylinder' or 'pulse'), nx, ny, Ma, steps and storage ('f32' or
    'f16s'), half of each kind and storage."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, n_jobs))
    jobs = []
    for j in range(n_jobs):
        nx = int(rng.integers(side_range[0], side_range[1] + 1))
        ny = int(rng.integers(side_range[0], side_range[1] + 1))
        jobs.append(dict(
            id=j, arrival=float(t[j]),
            kind="cylinder" if rng.uniform() < 0.5 else "pulse",
            nx=nx, ny=ny, ma=float(rng.uniform(*ma_range)),
            steps=max(2, int(int(rng.integers(step_range[0], step_range[1] + 1)) * step_scale)),
            storage="f32" if rng.uniform() < 0.5 else "f16s",
            seed=int(rng.integers(0, 2 ** 31)),
        ))
    return jobs
