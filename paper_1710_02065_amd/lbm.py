"""Python binding of the C ABI in include/lbm.h (liblbm_hip.so).

Argument marshalling only: every step of the method runs in the HIP kernels
of the shared library.  Device memory comes from torch tensors (their
data_ptr()), and work goes to the stream given in the configuration
(torch.cuda.current_stream().cuda_stream by default in `Simulation`).  If the
library has not been built, importing this module raises: there is no CPU
fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")

LBM_D2Q9, LBM_D3Q19, LBM_D3Q27 = 9, 19, 27
LBM_F64, LBM_F32, LBM_F32S, LBM_F16S, LBM_M64, LBM_M32 = 0, 1, 2, 3, 4, 5
LBM_PERIODIC, LBM_FREESLIP, LBM_OUTFLOW, LBM_HALO = 0, 1, 2, 3
LBM_FLUID, LBM_SOLID, LBM_INLET = 0, 1, 2
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE, LBM_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
LBM_ALLOW_HIGH_MA, LBM_NO_GRAPH, LBM_FULL_ORDER, LBM_SPONGE_FIELD = 0x1, 0x2, 0x4, 0x8
LBM_BGK, LBM_MRT = 0x10, 0x20
LBM_MAX_LEVELS = 5
LBM_NOALLOC_MAX_JOBS = 256

STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f32s": LBM_F32S, "f16s": LBM_F16S,
           "m64": LBM_M64, "m32": LBM_M32}
STORAGE_BYTES = {LBM_F64: 8, LBM_F32: 4, LBM_F32S: 4, LBM_F16S: 2, LBM_M64: 8, LBM_M32: 4}

# every symbol the header declares
EXPORTS = ["lbm_config_init", "lbm_required_bytes", "lbm_create", "lbm_bind_memory",
           "lbm_init", "lbm_step", "lbm_sync", "lbm_time", "lbm_updates_per_step",
           "lbm_level_shape",
           "lbm_moments", "lbm_probe", "lbm_accumulate", "lbm_force", "lbm_totals", "lbm_set_sponge",
           "lbm_get_populations", "lbm_set_populations", "lbm_set_time", "lbm_interface_bytes",
           "lbm_get_interface", "lbm_set_interface",
           "lbm_step_batch", "lbm_step_batch_noalloc", "lbm_autotune", "lbm_halo_buffers", "lbm_halo_exchange",
           "lbm_destroy", "lbm_lattice_table", "lbm_last_error"]


class lbm_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("lattice", C.c_int32), ("storage", C.c_int32),
        ("device", C.c_int32),
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("tau", C.c_double), ("rho0", C.c_double), ("ma", C.c_double),
        ("u_dir", C.c_double * 3),
        ("face_bc", C.c_int32 * 6), ("sponge_width", C.c_int32 * 6),
        ("chi_max", C.c_double), ("rho_ref", C.c_double), ("u_ref", C.c_double * 3),
        ("refine_lo", C.c_int64 * 3), ("refine_hi", C.c_int64 * 3),
        ("seed", C.c_uint64), ("inlet_noise", C.c_double),
        ("stream", C.c_void_p), ("flags", C.c_uint32), ("block", C.c_uint32),
        ("nest_count", C.c_int32), ("nest_reserved", C.c_int32),
        ("nest_lo", (C.c_int64 * 3) * (LBM_MAX_LEVELS - 2)),
        ("nest_hi", (C.c_int64 * 3) * (LBM_MAX_LEVELS - 2)),
    ]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbm error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbm_hip.so is not built (run __graft_entry__.build() or "
                              "python paper_1710_02065_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64 = C.c_void_p, C.c_void_p, C.c_int64
        cfgp = C.POINTER(lbm_config)
        L.lbm_config_init.argtypes = [cfgp]
        L.lbm_config_init.restype = None
        L.lbm_required_bytes.argtypes = [cfgp]
        L.lbm_required_bytes.restype = C.c_size_t
        L.lbm_create.argtypes = [cfgp, C.POINTER(vp)]
        L.lbm_bind_memory.argtypes = [vp, vp, C.c_size_t]
        L.lbm_init.argtypes = [vp, C.c_int, dp, dp, dp, vp]
        L.lbm_step.argtypes = [vp, i64]
        L.lbm_sync.argtypes = [vp]
        L.lbm_time.argtypes = [vp]
        L.lbm_time.restype = i64
        L.lbm_updates_per_step.argtypes = [vp]
        L.lbm_updates_per_step.restype = i64
        L.lbm_level_shape.argtypes = [vp, C.c_int, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.lbm_moments.argtypes = [vp, C.c_int, dp, dp]
        L.lbm_probe.argtypes = [vp, C.c_int, vp, C.c_int, dp]
        L.lbm_force.argtypes = [vp, C.c_int, dp]
        L.lbm_totals.argtypes = [vp, C.c_int, dp]
        L.lbm_set_sponge.argtypes = [vp, C.c_int, dp, dp, dp]
        L.lbm_accumulate.argtypes = [vp, C.c_int, dp, dp]
        L.lbm_get_populations.argtypes = [vp, C.c_int, dp]
        L.lbm_set_populations.argtypes = [vp, C.c_int, dp]
        L.lbm_set_time.argtypes = [vp, i64]
        L.lbm_interface_bytes.argtypes = [vp, C.c_int]
        L.lbm_interface_bytes.restype = C.c_size_t
        L.lbm_get_interface.argtypes = [vp, C.c_int, vp]
        L.lbm_set_interface.argtypes = [vp, C.c_int, vp]
        L.lbm_step_batch.argtypes = [C.POINTER(vp), C.POINTER(i64), C.c_int]
        L.lbm_step_batch_noalloc.argtypes = [C.POINTER(vp), C.POINTER(i64), C.c_int]
        L.lbm_autotune.argtypes = [vp, C.c_int]
        L.lbm_halo_buffers.argtypes = [vp, C.c_int, C.POINTER(vp), C.POINTER(vp),
                                       C.POINTER(C.c_size_t)]
        L.lbm_halo_exchange.argtypes = [C.POINTER(vp), C.c_int, C.c_int]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        L.lbm_lattice_table.argtypes = [C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.lbm_last_error.argtypes = []
        L.lbm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise LbmError(rc, lib().lbm_last_error().decode())
    return rc


def _ptr(t):
    """data_ptr of a tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- raw ABI --
def lbm_config_init():
    cfg = lbm_config()
    lib().lbm_config_init(C.byref(cfg))
    return cfg


def lbm_required_bytes(cfg):
    return int(lib().lbm_required_bytes(C.byref(cfg)))


def lbm_create(cfg):
    h = C.c_void_p()
    _check(lib().lbm_create(C.byref(cfg), C.byref(h)))
    return h


def lbm_bind_memory(ctx, buf, nbytes):
    return _check(lib().lbm_bind_memory(ctx, _ptr(buf), nbytes))


def lbm_init(ctx, level, rho=None, u=None, pi_neq=None, mask=None):
    return _check(lib().lbm_init(ctx, level, _ptr(rho), _ptr(u), _ptr(pi_neq), _ptr(mask)))


def lbm_step(ctx, n):
    return _check(lib().lbm_step(ctx, int(n)))


def lbm_sync(ctx):
    return _check(lib().lbm_sync(ctx))


def lbm_time(ctx):
    return int(lib().lbm_time(ctx))


def lbm_updates_per_step(ctx):
    return _check(int(lib().lbm_updates_per_step(ctx)))


def lbm_level_shape(ctx, level):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().lbm_level_shape(ctx, level, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def lbm_moments(ctx, level, rho_out, u_out):
    return _check(lib().lbm_moments(ctx, level, _ptr(rho_out), _ptr(u_out)))


def lbm_probe(ctx, level, cells, rho_out):
    return _check(lib().lbm_probe(ctx, level, _ptr(cells), int(cells.numel()), _ptr(rho_out)))


def lbm_accumulate(ctx, level, sum1, sum2):
    return _check(lib().lbm_accumulate(ctx, level, _ptr(sum1), _ptr(sum2)))


def lbm_force(ctx, level, out):
    return _check(lib().lbm_force(ctx, level, _ptr(out)))


def lbm_set_sponge(ctx, level, chi, rho_ref=None, u_ref=None):
    return _check(lib().lbm_set_sponge(ctx, level, _ptr(chi), _ptr(rho_ref), _ptr(u_ref)))


def lbm_totals(ctx, level, out):
    return _check(lib().lbm_totals(ctx, level, _ptr(out)))


def lbm_get_populations(ctx, level, out):
    return _check(lib().lbm_get_populations(ctx, level, _ptr(out)))


def lbm_set_populations(ctx, level, inp):
    return _check(lib().lbm_set_populations(ctx, level, _ptr(inp)))


def lbm_set_time(ctx, t):
    return _check(lib().lbm_set_time(ctx, int(t)))


def lbm_interface_bytes(ctx, level):
    n = int(lib().lbm_interface_bytes(ctx, level))
    if n == 0:
        raise LbmError(LBM_EINVAL, lib().lbm_last_error().decode())
    return n


def lbm_get_interface(ctx, level, out):
    return _check(lib().lbm_get_interface(ctx, level, _ptr(out)))


def lbm_set_interface(ctx, level, inp):
    return _check(lib().lbm_set_interface(ctx, level, _ptr(inp)))


def lbm_step_batch(ctxs, steps):
    n = len(ctxs)
    arr = (C.c_void_p * n)(*[c.value for c in ctxs])
    st = (C.c_int64 * n)(*[int(s) for s in steps])
    return _check(lib().lbm_step_batch(arr, st, n))


def lbm_step_batch_noalloc(ctxs, steps):
    n = len(ctxs)
    arr = (C.c_void_p * n)(*[c.value for c in ctxs])
    st = (C.c_int64 * n)(*[int(s) for s in steps])
    return _check(lib().lbm_step_batch_noalloc(arr, st, n))


def lbm_autotune(ctx, trials=3):
    return _check(lib().lbm_autotune(ctx, trials))


def lbm_halo_buffers(ctx, side):
    """(send, recv, bytes): device addresses of the halo buffers of side 0
    (low) or 1 (high) of the last axis."""
    send, recv, nb = C.c_void_p(), C.c_void_p(), C.c_size_t()
    _check(lib().lbm_halo_buffers(ctx, side, C.byref(send), C.byref(recv), C.byref(nb)))
    return send.value, recv.value, nb.value


def lbm_halo_exchange(ctxs, periodic):
    n = len(ctxs)
    arr = (C.c_void_p * n)(*[c.value for c in ctxs])
    return _check(lib().lbm_halo_exchange(arr, n, 1 if periodic else 0))


def lbm_destroy(ctx):
    lib().lbm_destroy(ctx)


def lbm_lattice_table(lattice):
    xi = (C.c_int32 * (3 * lattice))()
    w = (C.c_double * lattice)()
    _check(lib().lbm_lattice_table(lattice, xi, w))
    return np.array(xi[:], dtype=np.int64).reshape(lattice, 3), np.array(w[:])


def lbm_last_error():
    return lib().lbm_last_error().decode()


# ------------------------------------------------------------ convenience --
def make_config(lattice=LBM_D3Q19, shape=(64, 64, 64), tau=0.6, storage="f32", rho0=1.0,
                ma=0.0, u_dir=(1.0, 0.0, 0.0), face_bc=(LBM_PERIODIC,) * 6,
                sponge_width=(0,) * 6, chi_max=0.0, rho_ref=1.0, u_ref=(0.0, 0.0, 0.0),
                refine_lo=(0, 0, 0), refine_hi=(0, 0, 0), seed=0, inlet_noise=0.0,
                stream=None, flags=0, block=0, device=0, nest=()):
    """Configuration block.  refine_lo/hi: box of level 1 in level-0
    coordinates; nest: further boxes [(lo, hi), ...], box k in the node
    coordinates of level k + 1."""
    cfg = lbm_config_init()
    cfg.lattice = lattice
    cfg.storage = STORAGE[storage] if isinstance(storage, str) else storage
    cfg.device = device
    nx, ny, nz = (tuple(shape) + (1,))[:3]
    cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
    cfg.tau, cfg.rho0, cfg.ma = tau, rho0, ma
    cfg.u_dir[:] = list(u_dir)
    cfg.face_bc[:] = list(face_bc)
    cfg.sponge_width[:] = list(sponge_width)
    cfg.chi_max, cfg.rho_ref = chi_max, rho_ref
    cfg.u_ref[:] = list(u_ref)
    cfg.refine_lo[:] = list(refine_lo)
    cfg.refine_hi[:] = list(refine_hi)
    cfg.seed, cfg.inlet_noise = seed, inlet_noise
    cfg.stream = stream
    cfg.flags, cfg.block = flags, block
    nest = list(nest)
    if len(nest) > LBM_MAX_LEVELS - 2:
        raise ValueError("at most %d nested boxes" % (LBM_MAX_LEVELS - 2))
    cfg.nest_count = len(nest)
    for k, (lo, hi) in enumerate(nest):
        cfg.nest_lo[k][:] = (list(lo) + [0, 0, 0])[:3]
        cfg.nest_hi[k][:] = (list(hi) + [0, 0, 0])[:3]
    return cfg


class Simulation:
    """One context with torch-managed inputs and outputs.

    All arrays are torch tensors on the context's device (numpy inputs are
    copied there); results are float64 tensors in the layouts of the header.
    """

    def __init__(self, cfg=None, **kw):
        import torch
        self.torch = torch
        if cfg is None:
            kw.setdefault("stream", torch.cuda.current_stream().cuda_stream)
            cfg = make_config(**kw)
        self.cfg = cfg
        self.device = torch.device("cuda", cfg.device)
        self.ctx = lbm_create(cfg)
        self.q = cfg.lattice
        # bound now: module globals may already be gone when a late __del__
        # runs at interpreter exit
        self._destroy = lib().lbm_destroy

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self._destroy(ctx)
            self.ctx = None

    def close(self):
        self.__del__()

    def shape(self, level=0):
        return lbm_level_shape(self.ctx, level)

    def ncell(self, level=0):
        nx, ny, nz = self.shape(level)
        return nx * ny * nz

    def _dev(self, a, dtype):
        if a is None:
            return None
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype).contiguous()

    def init(self, rho=None, u=None, pi_neq=None, mask=None, level=0):
        t = self.torch
        N = self.ncell(level)
        rho = self._dev(rho, t.float64)
        if u is not None:
            u = self._dev(u, t.float64).reshape(-1, N)
            if u.shape[0] < 3:
                u = t.cat([u, t.zeros(3 - u.shape[0], N, dtype=t.float64, device=self.device)])
        pi_neq = self._dev(pi_neq, t.float64)
        mask = self._dev(mask, t.uint8)
        self._keep = (rho, u, pi_neq, mask)  # alive until the stream passes
        lbm_init(self.ctx, level, rho, u, pi_neq, mask)
        return self

    def step(self, n=1):
        lbm_step(self.ctx, n)
        return self

    def sync(self):
        return lbm_sync(self.ctx)

    @property
    def time(self):
        return lbm_time(self.ctx)

    @property
    def updates_per_step(self):
        return lbm_updates_per_step(self.ctx)

    def moments(self, level=0):
        t = self.torch
        N = self.ncell(level)
        rho = t.empty(N, dtype=t.float64, device=self.device)
        u = t.empty(3, N, dtype=t.float64, device=self.device)
        lbm_moments(self.ctx, level, rho, u)
        return rho, u

    def force(self, level=0, out=None):
        """Momentum-exchange force on the SOLID cells (3 FP64 on the
        device); `out` may be a 3-element slice of a longer series."""
        if out is None:
            out = self.torch.empty(3, dtype=self.torch.float64, device=self.device)
        lbm_force(self.ctx, level, out)
        return out

    def set_sponge(self, chi, rho_ref=None, u_ref=None, level=0):
        """Absorbing layer given per cell (needs LBM_SPONGE_FIELD): chi [N],
        rho_ref [N], u_ref [3][N]; host or device arrays."""
        t = self.torch
        chi = self._dev(chi, t.float64)
        rho_ref = self._dev(rho_ref, t.float64)
        u_ref = self._dev(u_ref, t.float64)
        if u_ref is not None:
            u_ref = u_ref.reshape(-1, self.ncell(level))
            if u_ref.shape[0] < 3:
                u_ref = t.cat([u_ref, t.zeros(3 - u_ref.shape[0], u_ref.shape[1],
                                              dtype=t.float64, device=self.device)])
            u_ref = u_ref.contiguous()
        lbm_set_sponge(self.ctx, level, chi, rho_ref, u_ref)
        return self

    def totals(self, level=0, out=None):
        """(sum of rho - rho0, momentum x, y, z) over the updated cells, 4
        FP64 on the device."""
        if out is None:
            out = self.torch.empty(4, dtype=self.torch.float64, device=self.device)
        lbm_totals(self.ctx, level, out)
        return out

    def accumulate(self, sum1, sum2=None, level=0):
        """Add rho - rho0 (and its square) of the current state to the
        device FP64 arrays sum1 (and sum2) of one entry per cell."""
        lbm_accumulate(self.ctx, level, sum1, sum2)

    def populations(self, level=0):
        t = self.torch
        out = t.empty(self.q, self.ncell(level), dtype=t.float64, device=self.device)
        lbm_get_populations(self.ctx, level, out)
        return out

    def set_populations(self, f, level=0):
        f = self._dev(f, self.torch.float64)
        self._keep_f = f
        lbm_set_populations(self.ctx, level, f)

    def checkpoint(self):
        """Device copies of everything a resume needs: the time, the
        populations of every level and the records of every refinement
        interface."""
        t = self.torch
        nlev = self.levels
        pops = [self.populations(l) for l in range(nlev)]
        recs = []
        for l in range(nlev - 1):
            buf = t.empty(lbm_interface_bytes(self.ctx, l), dtype=t.uint8, device=self.device)
            lbm_get_interface(self.ctx, l, buf)
            recs.append(buf)
        return dict(time=self.time, pops=pops, interfaces=recs)

    def restore(self, ck):
        """Resume from `checkpoint()` output (call after init of every level)."""
        for l, f in enumerate(ck["pops"]):
            self.set_populations(f, l)
        self._keep_ck = ck
        for l, buf in enumerate(ck["interfaces"]):
            lbm_set_interface(self.ctx, l, buf)
        lbm_set_time(self.ctx, ck["time"])
        return self

    @property
    def levels(self):
        refined = any(self.cfg.refine_lo[:]) or any(self.cfg.refine_hi[:])
        return 1 + (1 + self.cfg.nest_count if refined else 0)

    def probe(self, cells, level=0):
        t = self.torch
        cells = self._dev(cells, t.int64)
        out = t.empty(cells.numel(), dtype=t.float64, device=self.device)
        lbm_probe(self.ctx, level, cells, out)
        return out
