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
        L.ora_equilibrium_ex.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp]
        L.ora_noneq_ex.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.ora_collide_ex.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double,
                                     C.c_double, dp, dp]
        L.ora_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.ora_splitmix64.restype = C.c_uint64
        L.ora_sponge_chi.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64]
        L.ora_sponge_chi.restype = C.c_double
        L.ora_collide_mrt.argtypes = [dp, dp, dp]
        L.ora_sponge_sigma.argtypes = [C.c_double, C.c_double, C.c_double]
        L.ora_sponge_sigma.restype = C.c_double
        L.ora_init.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.ora_step.argtypes = [C.c_void_p, C.c_void_p, dp, dp, C.c_int64]
        L.ora_moments.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp]
        L.ora_sizeof_grid.restype = C.c_int
        L.ora_force.argtypes = [C.c_void_p, C.c_void_p, dp, dp]
        L.ora_step_ex.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, dp, dp, C.c_int64,
                                  dp, dp, dp]
        L.ora_sizeof_refined.restype = C.c_int
        L.ora_ref_roles.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_ref_fill_ring.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp, C.c_double,
                                        dp, dp, dp, C.c_double, dp]
        L.ora_ref_import.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp, dp]
        _lib = L
        assert L.ora_sizeof_grid() == C.sizeof(OraGrid), "ora_grid layout mismatch"
        assert L.ora_sizeof_refined() == C.sizeof(OraRefined), "ora_refined layout mismatch"
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
        ("seed", C.c_uint64), ("inlet_noise", C.c_double), ("full_order", C.c_int),
        ("levels", C.c_int),
        ("sp_chi", C.c_void_p), ("sp_rho", C.c_void_p), ("sp_u", C.c_void_p),
        ("collision", C.c_int),
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


# collision of FLUID cells: the regularized operator of eq. (optimizedLB),
# or the comparators of Sec. II.A: LBM-BGK (eq. standardLB) and LBM-MRT
# (D2Q9, Lallemand & Luo 2000)
COLLISIONS = {"rr": 0, "bgk": 1, "mrt": 2}


def collide_mrt(f, rates):
    """D2Q9 MRT collision of one cell with rates (s_e, s_eps, s_q, s_nu)."""
    f = _f64(f, 9)
    out = np.zeros(9)
    lib().ora_collide_mrt(_dp(f), _dp(_f64(rates, 4)), _dp(out))
    return out


def _check_full(q, full):
    if full and q not in (9, 27):
        raise ValueError("full recursive regularization needs D2Q9 or D3Q27")


def equilibrium(q, rho, u, full=False):
    """f^eqH(rho, u); full=True expands to every order the lattice resolves
    (default: third order)."""
    _check_full(q, full)
    out = np.zeros(q)
    u3 = _f64(list(u) + [0.0] * (3 - len(u)))
    if full:
        lib().ora_equilibrium_ex(q, 1, float(rho), _dp(u3), _dp(out))
    else:
        lib().ora_equilibrium(q, float(rho), _dp(u3), _dp(out))
    return out


def noneq(q, u, a2, full=False):
    """f^neqH(a2, u); a2 packed (xx, yy, zz, xy, xz, yz)."""
    _check_full(q, full)
    out = np.zeros(q)
    u3 = _f64(list(u) + [0.0] * (3 - len(u)))
    a2 = _f64(a2, 6)
    if full:
        lib().ora_noneq_ex(q, 1, _dp(u3), _dp(a2), _dp(out))
    else:
        lib().ora_noneq(q, _dp(u3), _dp(a2), _dp(out))
    return out


def collide(q, f, tau, chi=0.0, rho_ref=1.0, u_ref=(0.0, 0.0, 0.0), full=False):
    _check_full(q, full)
    f = _f64(f, q)
    out = np.zeros(q)
    ur = _f64(list(u_ref) + [0.0] * (3 - len(u_ref)))
    if full:
        lib().ora_collide_ex(q, 1, _dp(f), float(tau), float(chi), float(rho_ref), _dp(ur),
                             _dp(out))
    else:
        lib().ora_collide(q, _dp(f), float(tau), float(chi), float(rho_ref), _dp(ur), _dp(out))
    return out


def collide_bgk(q, f, tau, chi=0.0, rho_ref=1.0, u_ref=(0.0, 0.0, 0.0)):
    f = _f64(f, q)
    out = np.zeros(q)
    ur = _f64(list(u_ref) + [0.0] * (3 - len(u_ref)))
    lib().ora_collide_bgk(q, _dp(f), float(tau), float(chi), float(rho_ref), _dp(ur), _dp(out))
    return out


def sponge_sigma(s, s0, L):
    """Absorbing-layer profile of Sec. II.C at coordinate s across a layer
    from s0 to L (0 outside)."""
    return lib().ora_sponge_sigma(float(s), float(s0), float(L))


def circular_sponge(shape, center, r0, r1, chi_max):
    """chi per cell for a circular (2D) or spherical layer: the profile in
    the distance from `center`, from r0 to r1 (test input builder)."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 +
                (0.0 if nz == 1 else (z - center[2]) ** 2)).ravel()
    return np.array([chi_max * sponge_sigma(v, r0, r1) for v in r])


def splitmix64(seed, k):
    return int(lib().ora_splitmix64(C.c_uint64(seed), C.c_uint64(k)))


class Grid:
    """One regular grid advanced by the oracle.

    Parameters mirror the library's configuration: lattice q in {9, 19, 27},
    shape (nx, ny, nz) with nz = 1 in 2D, tau, rho0, inlet velocity u_in,
    per-face rules (x-, x+, y-, y+, z-, z+), sponge widths, chi_max and the
    sponge reference state, seed and inlet noise for inlet cells;
    full_order=True regularizes to every order the lattice resolves (D2Q9
    and D3Q27) instead of the third.
    """

    def __init__(self, q, nx, ny, nz=1, tau=0.6, rho0=1.0, u_in=(0.0, 0.0, 0.0),
                 face_bc=(PERIODIC,) * 6, sponge_width=(0,) * 6, chi_max=0.0,
                 rho_ref=1.0, u_ref=(0.0, 0.0, 0.0), seed=0, inlet_noise=0.0,
                 mask=None, level=0, full_order=False, levels=1, collision="rr"):
        _check_full(q, full_order)
        if collision not in COLLISIONS or (collision == "mrt" and q != 9) or \
                (collision != "rr" and full_order):
            raise ValueError("collision %r on D%dQ%d" % (collision, 2 if q == 9 else 3, q))
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
        g.full_order = 1 if full_order else 0
        g.levels = levels
        g.collision = COLLISIONS[collision]
        self.g = g
        self._sponge = None
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

    def set_sponge(self, chi, rho_ref=None, u_ref=None):
        """Absorbing layer given per cell: chi [N] (replaces the face
        profile), reference density [N] and velocity [3][N] (None: the
        constant references)."""
        N = self.N
        arrs = [np.ascontiguousarray(chi, dtype=np.float64).reshape(N),
                None if rho_ref is None else np.ascontiguousarray(rho_ref, dtype=np.float64).reshape(N),
                None if u_ref is None else np.ascontiguousarray(u_ref, dtype=np.float64).reshape(3, N)]
        self._sponge = arrs  # kept alive while the grid points at them
        self.g.sp_chi = arrs[0].ctypes.data
        self.g.sp_rho = None if arrs[1] is None else arrs[1].ctypes.data
        self.g.sp_u = None if arrs[2] is None else arrs[2].ctypes.data
        return self

    def chi(self, x, y, z=0):
        return lib().ora_sponge_chi(C.byref(self.g), x, y, z)

    def force(self):
        """Momentum-exchange force on the SOLID cells (3 components)."""
        F = np.zeros(3)
        lib().ora_force(C.byref(self.g), self._mask_ptr, _dp(self.f), _dp(F))
        return F


class OraRefined(C.Structure):
    _fields_ = [("c", OraGrid), ("f", OraGrid), ("lo", C.c_int64 * 3), ("hi", C.c_int64 * 3)]


NORMAL, IMPORT, COVERED = 0, 1, 2


def _u8p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class RefinedGrid:
    """Two-level 2:1 refinement (Sec. II.B) advanced by the oracle.

    The fine grid covers the closed coarse-node box [lo, hi] with half the
    spacing and half the time step (eq. convective); tau_f = (4 tau_c - 1)/2
    so the physical viscosity is the same on both levels.  One coarse step:
      1. coarse sweep of NORMAL nodes (records coarse pre-collision moments
         M_c(t+1));
      2. fine sweep of the non-RING nodes (fine time 2t -> 2t+1);
      3. RING <- cubic-in-space interpolation of (M_c(t) + M_c(t+1)) / 2;
      4. fine sweep (2t+1 -> 2t+2), recording fine pre-collision moments;
      5. RING <- interpolation of M_c(t+1);
      6. IMPORT coarse nodes <- filtered fine moments.
    """

    def __init__(self, q, nx, ny, nz, lo, hi, tau=0.6, rho0=1.0, u_in=(0.0, 0.0, 0.0),
                 face_bc=(PERIODIC,) * 6, sponge_width=(0,) * 6, chi_max=0.0, rho_ref=1.0,
                 u_ref=(0.0, 0.0, 0.0), seed=0, inlet_noise=0.0, mask=None, fine_mask=None,
                 full_order=False):
        d = 2 if q == 9 else 3
        lo = list(lo) + [0] * (3 - len(lo))
        hi = list(hi) + [0] * (3 - len(hi))
        fshape = [2 * (hi[a] - lo[a]) + 1 if a < d else 1 for a in range(3)]
        tau_f = (4.0 * tau - 1.0) / 2.0
        self.coarse = Grid(q, nx, ny, nz, tau=tau, rho0=rho0, u_in=u_in, face_bc=face_bc,
                           sponge_width=sponge_width, chi_max=chi_max, rho_ref=rho_ref,
                           u_ref=u_ref, seed=seed, inlet_noise=inlet_noise, mask=mask, level=0,
                           full_order=full_order)
        self.fine = Grid(q, *fshape, tau=tau_f, rho0=rho0, u_in=u_in,
                         face_bc=(OUTFLOW, OUTFLOW, OUTFLOW, OUTFLOW,
                                  OUTFLOW if d == 3 else PERIODIC, OUTFLOW if d == 3 else PERIODIC),
                         seed=seed, inlet_noise=inlet_noise, mask=fine_mask, level=1,
                         full_order=full_order)
        R = OraRefined()
        R.c = self.coarse.g
        R.f = self.fine.g
        R.lo[:] = lo
        R.hi[:] = hi
        self.R = R
        self.q, self.d = q, d
        self.crole = np.zeros(self.coarse.N, dtype=np.uint8)
        self.fring = np.zeros(self.fine.N, dtype=np.uint8)
        lib().ora_ref_roles(C.byref(R), _u8p(self.crole), _u8p(self.fring))
        self.cskip = (self.crole != NORMAL).astype(np.uint8)
        Nc, Nf = self.coarse.N, self.fine.N
        self.M_prev = [np.zeros(Nc), np.zeros((3, Nc)), np.zeros((6, Nc))]
        self.M_next = None
        self.mf = [np.zeros(Nf), np.zeros((3, Nf)), np.zeros((6, Nf))]
        self.inited = [False, False]
        self.t = 0

    def init(self, level, rho=None, u=None, pineq=None):
        g = self.coarse if level == 0 else self.fine
        g.init(rho, u, pineq)
        if level == 0:
            # coarse moments at t = 0 are the initial fields
            N = g.N
            self.M_prev[0][:] = g.g.rho0 if rho is None else np.asarray(rho, dtype=float).reshape(N)
            if u is None:
                self.M_prev[1][:] = np.array(g.g.u_in[:])[:, None]
            else:
                uu = np.asarray(u, dtype=float).reshape(-1, N)
                self.M_prev[1][:] = 0.0
                self.M_prev[1][: uu.shape[0]] = uu
            self.M_prev[2][:] = 0.0 if pineq is None else np.asarray(pineq, dtype=float).reshape(6, N)
            if self.d == 2:
                self.M_prev[1][2] = 0.0
                self.M_prev[2][[2, 4, 5]] = 0.0
        self.inited[level] = True
        if all(self.inited):
            self.M_next = [a.copy() for a in self.M_prev]
            self._fill_ring(self.M_prev, 1.0, self.M_prev, 0.0)
            self.t = 0
            self.coarse.t = 0
            self.fine.t = 0
        return self

    def _fill_ring(self, Ma, wa, Mb, wb):
        lib().ora_ref_fill_ring(C.byref(self.R), _u8p(self.fring), _dp(Ma[0]), _dp(Ma[1]),
                                _dp(Ma[2]), wa, _dp(Mb[0]), _dp(Mb[1]), _dp(Mb[2]), wb,
                                _dp(self.fine.f))

    def _sweep(self, g, skip, moments=None):
        out = np.empty_like(g.f)
        r, u, a2 = (None, None, None) if moments is None else moments
        lib().ora_step_ex(C.byref(g.g), g._mask_ptr, _u8p(skip), _dp(g.f), _dp(out), g.t + 1,
                          _dp(r), _dp(u), _dp(a2))
        g.f = out
        g.t += 1

    def step(self, n=1):
        for _ in range(n):
            self._sweep(self.coarse, self.cskip, self.M_next)
            self._sweep(self.fine, self.fring)
            self._fill_ring(self.M_prev, 0.5, self.M_next, 0.5)
            self._sweep(self.fine, self.fring, self.mf)
            self._fill_ring(self.M_next, 1.0, self.M_next, 0.0)
            lib().ora_ref_import(C.byref(self.R), _u8p(self.crole), _dp(self.mf[0]),
                                 _dp(self.mf[1]), _dp(self.mf[2]), _dp(self.coarse.f))
            self.M_prev = [a.copy() for a in self.M_next]
            self.t += 1
        return self


class MultiLevelGrid:
    """Nested 2:1 refinement with any number of levels: the two-level
    coupling of Sec. II.B applied at every interface of a chain of boxes
    (the paper's cylinder and jet setups use four and five levels).

    Level l+1 covers the closed node box boxes[l] = (lo, hi) of level l with
    half its spacing and half its time step; tau_(l+1) = (4 tau_l - 1) / 2.
    Each level's outer shell is RING (from its parent), and the shell of
    [lo+1, hi-1] of its child's box IMPORT (from the child), deeper nodes
    COVERED.  One step of level l, recursively (eq. convective at each
    interface):
      1. sweep level l, recording its pre-collision moments M_l(t+1);
      2. if l has a child: step the child; RING(child) <- interpolation of
         (M_l(t) + M_l(t+1)) / 2; step the child; RING(child) <-
         interpolation of M_l(t+1); IMPORT(l) <- filtered child moments.
    With one box this is exactly RefinedGrid's schedule.
    """

    def __init__(self, q, nx, ny, nz, boxes, tau=0.6, rho0=1.0, u_in=(0.0, 0.0, 0.0),
                 face_bc=(PERIODIC,) * 6, sponge_width=(0,) * 6, chi_max=0.0, rho_ref=1.0,
                 u_ref=(0.0, 0.0, 0.0), seed=0, inlet_noise=0.0, masks=None,
                 full_order=False):
        d = 2 if q == 9 else 3
        nl = len(boxes) + 1
        masks = list(masks) if masks is not None else [None] * nl
        masks += [None] * (nl - len(masks))
        self.q, self.d, self.nlevels = q, d, nl
        self.grids = [Grid(q, nx, ny, nz, tau=tau, rho0=rho0, u_in=u_in, face_bc=face_bc,
                           sponge_width=sponge_width, chi_max=chi_max, rho_ref=rho_ref,
                           u_ref=u_ref, seed=seed, inlet_noise=inlet_noise, mask=masks[0],
                           level=0, full_order=full_order, levels=nl)]
        self.pairs = []
        t = tau
        for l, (lo, hi) in enumerate(boxes):
            lo = list(lo) + [0] * (3 - len(lo))
            hi = list(hi) + [0] * (3 - len(hi))
            shape = [2 * (hi[a] - lo[a]) + 1 if a < d else 1 for a in range(3)]
            t = (4.0 * t - 1.0) / 2.0
            zf = OUTFLOW if d == 3 else PERIODIC
            g = Grid(q, *shape, tau=t, rho0=rho0, u_in=u_in,
                     face_bc=(OUTFLOW, OUTFLOW, OUTFLOW, OUTFLOW, zf, zf), seed=seed,
                     inlet_noise=inlet_noise, mask=masks[l + 1], level=l + 1,
                     full_order=full_order, levels=nl)
            self.grids.append(g)
            R = OraRefined()
            R.c = self.grids[l].g
            R.f = g.g
            R.lo[:] = lo
            R.hi[:] = hi
            self.pairs.append(R)
        # roles: crole[l] from level l's child box, ring[l] on level l's shell
        self.crole = [np.zeros(g.N, dtype=np.uint8) for g in self.grids]
        self.ring = [np.zeros(g.N, dtype=np.uint8) for g in self.grids]
        for l, R in enumerate(self.pairs):
            lib().ora_ref_roles(C.byref(R), _u8p(self.crole[l]), _u8p(self.ring[l + 1]))
        self.skip = [((self.crole[l] != NORMAL) | (self.ring[l] != 0)).astype(np.uint8)
                     for l in range(nl)]
        self.mom = [[np.zeros(g.N), np.zeros((3, g.N)), np.zeros((6, g.N))] for g in self.grids]
        self.M_prev = [None] * nl
        self.inited = [False] * nl
        self.t = 0

    def init(self, level, rho=None, u=None, pineq=None):
        g = self.grids[level]
        g.init(rho, u, pineq)
        N = g.N
        M = [np.zeros(N), np.zeros((3, N)), np.zeros((6, N))]
        M[0][:] = g.g.rho0 if rho is None else np.asarray(rho, dtype=float).reshape(N)
        if u is None:
            M[1][:] = np.array(g.g.u_in[:])[:, None]
        else:
            uu = np.asarray(u, dtype=float).reshape(-1, N)
            M[1][: uu.shape[0]] = uu
        if pineq is not None:
            M[2][:] = np.asarray(pineq, dtype=float).reshape(6, N)
        if self.d == 2:
            M[1][2] = 0.0
            M[2][[2, 4, 5]] = 0.0
        self.M_prev[level] = M
        self.inited[level] = True
        if all(self.inited):
            for l in range(1, self.nlevels):
                self._fill_ring(l - 1, self.M_prev[l - 1], 1.0, self.M_prev[l - 1], 0.0)
            self.t = 0
            for gg in self.grids:
                gg.t = 0
        return self

    def _fill_ring(self, l, Ma, wa, Mb, wb):
        """RING of level l+1 from level-l moments wa Ma + wb Mb."""
        lib().ora_ref_fill_ring(C.byref(self.pairs[l]), _u8p(self.ring[l + 1]), _dp(Ma[0]),
                                _dp(Ma[1]), _dp(Ma[2]), wa, _dp(Mb[0]), _dp(Mb[1]),
                                _dp(Mb[2]), wb, _dp(self.grids[l + 1].f))

    def _advance(self, l):
        g = self.grids[l]
        out = np.empty_like(g.f)
        r, u, a2 = self.mom[l]
        lib().ora_step_ex(C.byref(g.g), g._mask_ptr, _u8p(self.skip[l]), _dp(g.f), _dp(out),
                          g.t + 1, _dp(r), _dp(u), _dp(a2))
        g.f = out
        g.t += 1
        if l + 1 < self.nlevels:
            # cells the sweep skipped keep their M(t) values in M(t+1)
            nxt = [a.copy() for a in self.M_prev[l]]
            upd = self.skip[l] == 0
            for a, m in zip(nxt, self.mom[l]):
                a[..., upd] = m[..., upd]
            self._advance(l + 1)
            self._fill_ring(l, self.M_prev[l], 0.5, nxt, 0.5)
            self._advance(l + 1)
            self._fill_ring(l, nxt, 1.0, nxt, 0.0)
            mf = self.mom[l + 1]
            lib().ora_ref_import(C.byref(self.pairs[l]), _u8p(self.crole[l]), _dp(mf[0]),
                                 _dp(mf[1]), _dp(mf[2]), _dp(g.f))
            self.M_prev[l] = nxt

    def step(self, n=1):
        for _ in range(n):
            self._advance(0)
            self.t += 1
        return self
