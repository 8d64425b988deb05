"""ctypes wrapper around the FP64 CPU oracle (liblbm_oracle.so).

Test infrastructure: the GPU library never imports this module.  Arrays are
numpy float64, populations in [q][N] order with N = nz*ny*nx, x fastest.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

PERIODIC, FREESLIP, OUTFLOW = 0, 1, 2
FLUID, SOLID, INLET = 0, 1, 2
CS2 = 1.0 / 3.0

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.ora_lattice_info.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), dp, C.POINTER(C.c_int)]
        L.ora_equilibrium.argtypes = [C.c_int, C.c_double, dp, dp]
        L.ora_noneq.argtypes = [C.c_int, dp, dp, dp]
        L.ora_collide.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, dp, dp]
        L.ora_collide_bgk.argtypes = L.ora_collide.argtypes
        L.ora_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.ora_splitmix64.restype = C.c_uint64
        L.ora_sponge_chi.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64]
        L.ora_sponge_chi.restype = C.c_double
        L.ora_init.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.ora_step.argtypes = [C.c_void_p, C.c_void_p, dp, dp, C.c_int64]
        L.ora_moments.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp]
        L.ora_sizeof_grid.restype = C.c_int
        _lib = L
        assert L.ora_sizeof_grid() == C.sizeof(OraGrid), "ora_grid layout mismatch"
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


class OraGrid(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("level", C.c_int),
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("u_in", C.c_double * 3),
        ("face_bc", C.c_int * 6), ("sponge_width", C.c_int * 6),
        ("chi_max", C.c_double), ("rho_ref", C.c_double), ("u_ref", C.c_double * 3),
        ("seed", C.c_uint64), ("inlet_noise", C.c_double),
    ]


def lattice(q):
    """(xi [q,3] int, w [q], opp [q]) from the oracle's own table."""
    L = lib()
    xi = (C.c_int * (3 * q))()
    w = (C.c_double * q)()
    opp = (C.c_int * q)()
    qq, dd = C.c_int(), C.c_int()
    if L.ora_lattice_info(q, C.byref(qq), C.byref(dd), xi, w, opp) != 0:
        raise ValueError("unknown lattice %r" % q)
    return (np.array(xi[:], dtype=np.int64).reshape(q, 3), np.array(w[:]),
            np.array(opp[:], dtype=np.int64))


def equilibrium(q, rho, u):
    out = np.zeros(q)
    u3 = _f64(list(u) + [0.0] * (3 - len(u)))
    lib().ora_equilibrium(q, float(rho), _dp(u3), _dp(out))
    return out


def noneq(q, u, a2):
    """a2 packed (xx, yy, zz, xy, xz, yz)."""
    out = np.zeros(q)
    u3 = _f64(list(u) + [0.0] * (3 - len(u)))
    a2 = _f64(a2, 6)
    lib().ora_noneq(q, _dp(u3), _dp(a2), _dp(out))
    return out


def collide(q, f, tau, chi=0.0, rho_ref=1.0, u_ref=(0.0, 0.0, 0.0)):
    f = _f64(f, q)
    out = np.zeros(q)
    ur = _f64(list(u_ref) + [0.0] * (3 - len(u_ref)))
    lib().ora_collide(q, _dp(f), float(tau), float(chi), float(rho_ref), _dp(ur), _dp(out))
    return out


def collide_bgk(q, f, tau, chi=0.0, rho_ref=1.0, u_ref=(0.0, 0.0, 0.0)):
    f = _f64(f, q)
    out = np.zeros(q)
    ur = _f64(list(u_ref) + [0.0] * (3 - len(u_ref)))
    lib().ora_collide_bgk(q, _dp(f), float(tau), float(chi), float(rho_ref), _dp(ur), _dp(out))
    return out


def splitmix64(seed, k):
    return int(lib().ora_splitmix64(C.c_uint64(seed), C.c_uint64(k)))


class Grid:
    """One regular grid advanced by the oracle.

    Parameters mirror the library's configuration: lattice q in {9, 19, 27},
    shape (nx, ny, nz) with nz = 1 in 2D, tau, rho0, inlet velocity u_in,
    per-face rules (x-, x+, y-, y+, z-, z+), sponge widths, chi_max and the
    sponge reference state, seed and inlet noise for inlet cells.
    """

    def __init__(self, q, nx, ny, nz=1, tau=0.6, rho0=1.0, u_in=(0.0, 0.0, 0.0),
                 face_bc=(PERIODIC,) * 6, sponge_width=(0,) * 6, chi_max=0.0,
                 rho_ref=1.0, u_ref=(0.0, 0.0, 0.0), seed=0, inlet_noise=0.0,
                 mask=None, level=0):
        self.q = q
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        g = OraGrid()
        g.lattice, g.level = q, level
        g.nx, g.ny, g.nz = nx, ny, nz
        g.tau, g.rho0 = tau, rho0
        g.u_in[:] = list(u_in) + [0.0] * (3 - len(u_in))
        g.face_bc[:] = list(face_bc)
        g.sponge_width[:] = list(sponge_width)
        g.chi_max, g.rho_ref = chi_max, rho_ref
        g.u_ref[:] = list(u_ref) + [0.0] * (3 - len(u_ref))
        g.seed, g.inlet_noise = seed, inlet_noise
        self.g = g
        self.mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        if self.mask is not None:
            assert self.mask.size == self.N
        self.f = np.zeros((q, self.N))
        self.t = 0

    @property
    def _mask_ptr(self):
        return None if self.mask is None else self.mask.ctypes.data_as(C.c_void_p)

    def init(self, rho=None, u=None, pineq=None):
        N = self.N
        r = None if rho is None else _f64(rho, N)
        uu = None
        if u is not None:
            u = np.asarray(u, dtype=np.float64).reshape(-1, N)
            uu = np.zeros((3, N))
            uu[: u.shape[0]] = u
        p = None if pineq is None else _f64(pineq, 6 * N)
        lib().ora_init(C.byref(self.g), _dp(r), _dp(uu), _dp(p), _dp(self.f))
        self.t = 0
        return self

    def set_populations(self, f):
        self.f = _f64(f, self.q * self.N).reshape(self.q, self.N).copy()

    def step(self, n=1):
        out = np.empty_like(self.f)
        for _ in range(n):
            lib().ora_step(C.byref(self.g), self._mask_ptr, _dp(self.f), _dp(out), self.t + 1)
            self.f, out = out, self.f
            self.t += 1
        return self

    def moments(self):
        rho = np.empty(self.N)
        u = np.empty((3, self.N))
        lib().ora_moments(C.byref(self.g), self._mask_ptr, _dp(self.f), _dp(rho), _dp(u))
        return rho, u

    def chi(self, x, y, z=0):
        return lib().ora_sponge_chi(C.byref(self.g), x, y, z)
