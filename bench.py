"""Benchmark of the fused pull-stream + Hermite-regularized collision sweep.

Workload (the headline): D3Q19, 256^3 periodic cells, 3D Taylor-Green
vortex at U = 0.1 cs plus a Gaussian acoustic pulse (1e-3 rho0, sigma 8
cells), tau = 0.52, FP32 arithmetic with FP32 population storage; synthetic
fields generated on the host, resident in HBM before timing.  One step is one
sweep over the whole grid (pull, moments, regularized collision, store).

Prints one JSON line: MLUPS (whole job), the HBM roofline of the sweep kernel
(algorithmic bytes 2 q sizeof(storage) per cell update over the kernel time
measured with HIP events on the launch stream), the other storage forms
(FP16-shifted, FP32-shifted, FP64, and the moment storages M32 / M64 that
keep 10 moments per cell instead of 19 populations) with their speedups, the
precision of each FP32 / 16-bit form against the FP64 build (which matches
the oracle to 1e-12), and the FP64 CPU oracle timed on the host cores on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# workgroup size of the timed headline sweep (D3Q19 FP32), fixed so that the
# committed kernel trace and counters describe the launch this run times
HEADLINE_BLOCK = 256
METRIC = "MLUPS & % HBM roofline (D3Q19 256³); p50/p99 latency, batched serving"
# sources each profiled kernel is compiled from
SOURCES = {"k_sweep": ["kernels.hip", "kernels.hpp", "lattice.hpp"],
           "k_msweep": ["msweep.hip", "kernels.hpp", "lattice.hpp"]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(kernel="k_sweep"):
    h = hashlib.sha256()
    for s in SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1710_02065_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % name)
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                d[k.strip()] = v.strip()
    if d.get("kernel_hash") != kernel_hash(name.split("_d3q")[0]):
        return None
    return int(d["bytes_per_launch"])


def run_gpu(lbm, torch, storage, n, steps, warmup, fields, block=0, lattice=19, flags=0,
            windows=1):
    """Initialise, warm up, pick the workgroup size with the library's
    autotuner (unless one is given), then time `windows` windows of `steps`
    steps each with HIP events on the launch stream; returns the simulation,
    the median window in ms and every window."""
    rho, u = fields
    sim = lbm.Simulation(lattice=lattice, shape=(n, n, n), tau=0.52, storage=storage,
                         block=block, flags=flags)
    sim.init(rho, u)
    sim.step(warmup)
    sim.sync()
    sim.block = block or lbm.lbm_autotune(sim.ctx, 2)
    sim.step(2)
    sim.sync()
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(windows):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        sim.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        times.append(t0.elapsed_time(t1))
    sim.sync()
    return sim, float(np.median(times)), times


def copy_bandwidth(torch, nbytes=2 ** 31, reps=10):
    """Device-to-device copy rate (bytes read + written per second) of a
    plain 2 GiB torch copy, timed with HIP events: the practical ceiling
    reported beside the 8 TB/s spec peak."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(gbs, 1)


def pressure_error(sim, ref_rho, rho0=1.0):
    r, u = sim.moments()
    cs2 = 1.0 / 3.0
    p = cs2 * (r - rho0)
    pref = cs2 * (ref_rho - rho0)
    return float(((p - pref).norm() / pref.norm()).item()), r, u


def anchor_states(lbm, torch, n, fields, steps, storages=("f64", "f32", "f16s", "m32")):
    """The headline workload stepped `steps` times from the same fields in
    each storage; host copies of rho and u (and of the FP64 build's
    populations) for the comparison with the oracle in the CPU leg."""
    out = {}
    for st in storages:
        sim = lbm.Simulation(lattice=19, shape=(n, n, n), tau=0.52, storage=st)
        sim.init(*fields)
        sim.step(steps)
        r, u = sim.moments()
        out[st] = dict(rho=r.cpu().numpy(), u=u.cpu().numpy())
        if st == "f64":
            out[st]["pops"] = sim.populations().cpu().numpy()
        sim.sync()
        del sim, r, u
        torch.cuda.empty_cache()
    return out


def cpu_baseline(n, steps, anchors=None):
    """The FP64 oracle on the host cores over the same 256^3 workload:
    initialisation, then `steps` timed whole-grid steps.  Its final state is
    also the direct anchor of the GPU storages stepped as many times from the
    same fields (`anchors`, from anchor_states): relative L2 error of the
    acoustic pressure p' = cs^2 (rho - rho0) and of u, and for the FP64 build
    the normwise population error."""
    import oracle as O
    from paper_1710_02065_amd import workloads as W
    U = 0.1 / math.sqrt(3)
    rho, u = W.taylor_green_3d(n, U, pulse_amp=1e-3, pulse_sigma=8.0)
    g = O.Grid(19, n, n, n, tau=0.52).init(rho, u)
    del rho, u
    t0 = time.perf_counter()
    g.step(steps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    cores = min(threads, avail) if threads > 0 else avail
    res = dict(value=round(g.N * steps / dt / 1e6, 3), unit="MLUPS", cores=cores, kind="oracle",
               sample="FP64 oracle, D3Q19 %d^3 Taylor-Green + pulse, %d whole-grid steps "
                      "(%.1f s) after initialisation" % (n, steps, dt))
    if anchors:
        r_o, u_o = g.moments()
        p_o = (r_o - 1.0) / 3.0
        rows = {}
        for st, a in anchors.items():
            row = dict(p_rel_l2=float(np.linalg.norm((a["rho"] - 1.0) / 3.0 - p_o)
                                      / np.linalg.norm(p_o)),
                       u_rel_l2=float(np.linalg.norm(a["u"] - u_o) / np.linalg.norm(u_o)))
            if "pops" in a:
                row["populations_normwise"] = float(np.abs(a["pops"] - g.f).max()
                                                    / np.abs(g.f).max())
            rows[st] = row
        res["anchor_vs_gpu"] = dict(
            steps=steps, errors=rows,
            note="GPU storages against this oracle run, same fields and steps, whole grid")
    return res


def precision_study(lbm, torch, n, fields, horizons):
    """FP32, FP32-shifted, FP16-shifted and FP32-moment storage run side by side with the
    FP64 build (which matches the oracle to 1e-12) on the headline workload;
    relative L2 error of the acoustic pressure p' = cs^2 (rho - rho0) and of
    u at each horizon."""
    sims = {}
    for st in ("f64", "f32", "f32s", "f16s", "m32"):
        sims[st] = lbm.Simulation(lattice=19, shape=(n, n, n), tau=0.52, storage=st)
        sims[st].init(*fields)
    out = {}
    done = 0
    for T in horizons:
        for sim in sims.values():
            sim.step(T - done)
        done = T
        r64, u64 = sims["f64"].moments()
        p64 = (r64 - 1.0) / 3.0
        row = {}
        for st in ("f32", "f32s", "f16s", "m32"):
            r, u = sims[st].moments()
            row[st] = dict(p_rel_l2=float((((r - 1.0) / 3.0 - p64).norm() / p64.norm()).item()),
                           u_rel_l2=float(((u - u64).norm() / u64.norm()).item()))
        out[str(T)] = row
    for sim in sims.values():
        sim.sync()
    del sims
    torch.cuda.empty_cache()
    return out


def time_steps(sim, torch, steps):
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    sim.step(steps)
    b.record(stream)
    torch.cuda.synchronize()
    sim.sync()
    return a.elapsed_time(b)


def slab_rehearsal(lbm, torch, n, fields, steps, headline_mlups, k=8):
    """The headline grid spread over k GPUs in z-slabs, on this one GPU.

    share: one GPU's n x n x (n/k) slab with both z faces cut (LBM_HALO),
    its sweep timed alone (halo pack fused into it) and then with its halos
    moved each step (here to itself: two device copies of the crossing
    populations, the stand-in for grouped send/recv over xGMI);
    all_slabs: the k slabs stepped in lockstep on this GPU with the exchange
    between steps, against the undivided grid's throughput."""
    from paper_1710_02065_amd.slabs import Slabs
    rho, u = fields
    nz = n // k
    cells = n * n * nz
    sim = lbm.Simulation(lattice=19, shape=(n, n, nz), tau=0.52, storage="f32",
                         face_bc=(0, 0, 0, 0, lbm.LBM_HALO, lbm.LBM_HALO))
    sim.init(rho[:cells].contiguous(), u[:, :cells].contiguous())
    ring = [sim.ctx]
    for _ in range(20):
        sim.step(1)
        lbm.lbm_halo_exchange(ring, True)
    sim.sync()
    sim.block = lbm.lbm_autotune(sim.ctx, 2)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def sweep_only():
        sim.step(1)

    def sweep_and_exchange():
        sim.step(1)
        lbm.lbm_halo_exchange(ring, True)

    ms_sweep = timed(sweep_only, steps)
    ms_both = timed(sweep_and_exchange, steps)
    sim.sync()
    _, _, hb = lbm.lbm_halo_buffers(sim.ctx, 0)
    share = dict(shape=[n, n, nz], mlups=round(cells / (ms_sweep * 1e3), 1),
                 hbm_gbs=round(152 * cells / (ms_sweep / 1e3) / 1e9, 1),
                 sweep_us=round(ms_sweep * 1e3, 2),
                 exchange_us=round((ms_both - ms_sweep) * 1e3, 2),
                 halo_bytes_per_cut_and_direction=hb, workgroup=sim.block)
    del sim
    torch.cuda.empty_cache()
    sl = Slabs(k, (n, n, n), lattice=19, tau=0.52, storage="f32")
    sl.init(rho, u)
    sl.step(10)
    sl.sync()
    ms_all = timed(lambda: sl.step(1), max(steps // k, 20))
    sl.sync()
    sl.close()
    del sl
    torch.cuda.empty_cache()
    mlups_all = n ** 3 / (ms_all * 1e3)
    return {"workload": "D3Q19 %d^3 FP32 (the headline grid) in %d z-slabs of %d planes"
                        % (n, k, nz),
            "share": share,
            "all_slabs_on_one_gpu": dict(mlups=round(mlups_all, 1),
                                         vs_undivided=round(mlups_all / headline_mlups, 3)),
            "note": "one GPU's share timed alone; a k-GPU run would step the k shares "
                    "concurrently with the exchange on the links (not measured here)"}


def other_configs(lbm, torch, steps, shedding_steps,
                  which=("c1", "c2", "cylinder_levels", "stability", "c4")):
    """Full-size runs of the other single-GPU configurations (not the
    headline): the D2Q9 Taylor-Green and cylinder channel, the cylinder on
    four nested levels, the stability study and the D3Q27 jet with a 2:1
    block; `which` selects them."""
    from paper_1710_02065_amd import workloads as W
    res = {}
    if "c1" in which:
        # D2Q9 128^2 periodic Taylor-Green in FP64 (U = 0.05, tau 0.6, 1000
        # steps): fitted viscosity against cs^2 (tau - 1/2) = 1/30, mass and
        # momentum drift; a latency-bound size, timed for completeness
        n1, U1, tau1, T1 = 128, 0.05, 0.6, 1000
        rho1, u1, S1 = W.taylor_green_2d(n1, U1)
        sim = lbm.Simulation(lattice=9, shape=(n1, n1, 1), tau=tau1, storage="f64")
        sim.init(rho1, u1, -2.0 * rho1 * tau1 / 3.0 * S1)
        mode = torch.from_numpy(W.taylor_green_mode_2d(n1)).cuda()
        t0 = sim.totals().cpu().numpy()
        sim.step(100)
        a0 = float((sim.moments()[1][0] @ mode) / (mode @ mode))
        ms1 = time_steps(sim, torch, T1 - 100)
        a1 = float((sim.moments()[1][0] @ mode) / (mode @ mode))
        t1 = sim.totals().cpu().numpy()
        sim.sync()
        k1 = 2 * math.pi / n1
        nu_fit = -math.log(a1 / a0) / (2 * k1 * k1 * (T1 - 100))
        res["d2q9_taylor_green_128_f64"] = dict(
            nu_fit=nu_fit, nu_theory=1.0 / 30.0, nu_rel_error=nu_fit * 30.0 - 1.0,
            mass_drift=float(abs(t1[0] - t0[0]) / (n1 * n1)),
            momentum_drift=float(np.abs(t1[1:] - t0[1:]).max() / (n1 * n1)),
            mlups=round(n1 * n1 * (T1 - 100) / (ms1 * 1e3), 1), steps=T1,
            note="drifts per cell; 16k cells cannot fill the GPU")
        del sim
    if "c2" in which:
        # D2Q9 2048 x 1024 channel, cylinder D = 100 at (400, 512), Ma 0.2, Re 150
        nx, ny, D = 2048, 1024, 100
        U = 0.2 * math.sqrt(1.0 / 3.0)
        sim = lbm.Simulation(lattice=9, shape=(nx, ny, 1), tau=0.5 + 3 * U * D / 150, storage="f32",
                             ma=0.2, face_bc=(2, 2, 1, 1, 0, 0), sponge_width=(0, 128, 0, 0, 0, 0),
                             chi_max=0.2, rho_ref=1.0, u_ref=(U, 0, 0), seed=2)
        rho, u = W.uniform_perturbed((nx, ny, 1), U, (1, 0, 0), seed=2, rel_noise=1e-4, d=2)
        sim.init(rho, u, None, W.cylinder_mask(nx, ny, D, 400, 512))
        sim.step(64)
        sim.block = lbm.lbm_autotune(sim.ctx, 2)
        ms = time_steps(sim, torch, steps)
        N = nx * ny
        bytes_lup = 2 * 9 * 4 + 1
        res["d2q9_cylinder_2048x1024_f32"] = dict(
            mlups=round(N * steps / (ms * 1e3), 1), steps=steps, workgroup=sim.block,
            hbm_gbs=round(bytes_lup * N * steps / (ms / 1e3) / 1e9, 1),
            note="72 B/LUP populations + 1 B mask; 151 MB of state fits the 256 MB MALL")
        del sim
        torch.cuda.empty_cache()
        # the channel in FP32 against the FP64 build (equal to the oracle within
        # 1e-12 in the parity tests) after 2000 steps
        fields = {}
        for st in ("f64", "f32"):
            sv = lbm.Simulation(lattice=9, shape=(nx, ny, 1), tau=0.5 + 3 * U * D / 150,
                                storage=st, ma=0.2, face_bc=(2, 2, 1, 1, 0, 0),
                                sponge_width=(0, 128, 0, 0, 0, 0), chi_max=0.2, rho_ref=1.0,
                                u_ref=(U, 0, 0), seed=2)
            sv.init(rho, u, None, W.cylinder_mask(nx, ny, D, 400, 512))
            sv.step(2000)
            fields[st] = sv.moments()
            sv.sync()
            del sv
        (r64, u64), (r32, u32) = fields["f64"], fields["f32"]
        fluid = r64 != 0
        p64 = (r64 - 1.0)[fluid]
        res["d2q9_cylinder_2048x1024_f32_vs_f64_2000_steps"] = dict(
            p_rel_l2=float(((r32 - r64)[fluid]).norm() / p64.norm()),
            u_rel_l2=float((u32 - u64)[:, fluid].norm() / u64[:, fluid].norm()),
            u_max_abs=float((u32 - u64)[:, fluid].abs().max()))
        del fields, r64, u64, r32, u32
        torch.cuda.empty_cache()
        if shedding_steps:
            # the same channel run long enough for periodic shedding: C_L, St
            # and C_D by momentum exchange (Sec. III); walls 5 D from the body
            from paper_1710_02065_amd import cylinder_study
            w = min(60000, shedding_steps // 2)
            res["d2q9_cylinder_2048x1024_shedding"] = cylinder_study.run(
                steps=shedding_steps, window=w, acoustics=False,
                probe_cells=W.cylinder_probes(nx, ny, D, 400, 512), log=log)
            res["d2q9_cylinder_2048x1024_shedding"]["probes"] = (
                "p = cs^2 rho every 10 steps at r = 1.5, 2, 3, 4 D along 90 and 78.2 degrees")
            torch.cuda.empty_cache()
    if "cylinder_levels" in which:
        # the cylinder on four nested levels with a circular layer (the
        # arrangement of Sec. III): C_L, St, C_D, directivity, far-field decay
        from paper_1710_02065_amd import cylinder_levels
        res["d2q9_cylinder_four_levels"] = cylinder_levels.run(log=log)
        torch.cuda.empty_cache()
    if "stability" in which:
        # stability of the collision operators (Sec. II.A): smallest stable tau
        # on a D2Q9 128^2 thick shear layer at Ma 0.2
        from paper_1710_02065_amd import stability_study
        res["d2q9_shear_layer_stability"] = stability_study.run(n=128, ma=0.2, log=log)
        torch.cuda.empty_cache()
    if "c4" in which:
        # D3Q27 384 x 256 x 256 jet, inlet disc D = 20 at Ma 0.3 with 2 % noise,
        # Re 3600, 64-cell sponge on x+, y+-, z+-, 2:1 block [4,196]x[64,191]x[64,191]
        # The second run gives the outflow layer the round-jet similarity field
        # as its reference (Sec. IV), through the per-cell layer with the same
        # face profile.
        from paper_1710_02065_amd import layers
        shape = (384, 256, 256)
        Uj = 0.3 * math.sqrt(1.0 / 3.0)
        nu = Uj * 20 / 3600
        tau = 0.5 + 3 * nu
        lo, hi = (4, 64, 64), (196, 191, 191)
        widths = (0, 64, 64, 64, 64, 64)
        for name, field in (("d3q27_jet_384x256x256_refined_f32", False),
                            ("d3q27_jet_384x256x256_refined_f32_similarity_reference", True)):
            sim = lbm.Simulation(lattice=27, shape=shape, tau=tau, storage="f32", ma=0.3,
                                 face_bc=(2, 2, 2, 2, 2, 2), sponge_width=widths,
                                 chi_max=0.2, rho_ref=1.0, seed=4, inlet_noise=0.02,
                                 refine_lo=lo, refine_hi=hi,
                                 flags=lbm.LBM_SPONGE_FIELD if field else 0)
            sim.init(None, torch.zeros(3, shape[0] * shape[1] * shape[2], dtype=torch.float64,
                                       device="cuda"), None, W.jet_inlet_mask(*shape, D=20), level=0)
            fs = sim.shape(1)
            sim.init(None, torch.zeros(3, fs[0] * fs[1] * fs[2], dtype=torch.float64,
                                       device="cuda"), level=1)
            if field:
                rr, ur = layers.jet_reference(shape, 20.0, Uj)
                sim.set_sponge(layers.face_layer(shape, widths, 0.2), rr, ur, level=0)
                del rr, ur
            sim.step(8)
            js = max(steps // 10, 20)
            ms = time_steps(sim, torch, js)
            ups = sim.updates_per_step
            res[name] = dict(
                mlups=round(ups * js / (ms * 1e3), 1), coarse_steps=js, updates_per_coarse_step=ups,
                hbm_gbs=round(2 * 27 * 4 * ups * js / (ms / 1e3) / 1e9, 1),
                note="updates = swept coarse cells + 2 x swept fine cells per coarse step; "
                     "refined block starts 4 cells from the inlet face (coupling margin)"
                     + ("; per-cell layer (20 B more per layer cell) with the round-jet "
                        "similarity velocity as reference" if field else ""))
            del sim
            torch.cuda.empty_cache()
        # FP32 against the FP64 build (which the parity tests match to the
        # oracle within 1e-12 on reduced refined jets) after a short horizon,
        # per level, over the swept cells
        horizon = 100
        mom = {}
        for st in ("f64", "f32"):
            sim = lbm.Simulation(lattice=27, shape=shape, tau=tau, storage=st, ma=0.3,
                                 face_bc=(2, 2, 2, 2, 2, 2), sponge_width=widths,
                                 chi_max=0.2, rho_ref=1.0, seed=4, inlet_noise=0.02,
                                 refine_lo=lo, refine_hi=hi)
            for lev in (0, 1):
                ls = sim.shape(lev)
                sim.init(None, torch.zeros(3, ls[0] * ls[1] * ls[2], dtype=torch.float64,
                                           device="cuda"), None,
                         W.jet_inlet_mask(*shape, D=20) if lev == 0 else None, level=lev)
            sim.step(horizon)
            mom[st] = [sim.moments(lev) for lev in (0, 1)]
            sim.sync()
            del sim
            torch.cuda.empty_cache()
        err = {}
        for lev in (0, 1):
            (r64, u64), (r32, u32) = mom["f64"][lev], mom["f32"][lev]
            live = r64 != 0  # SOLID and COVERED cells report 0
            p64 = (r64 - 1.0)[live]
            err["level%d" % lev] = dict(
                p_rel_l2=float((r32 - r64)[live].norm() / p64.norm()),
                u_rel_l2=float((u32 - u64)[:, live].norm() / u64[:, live].norm()))
        res["d3q27_jet_384x256x256_refined_f32_vs_f64"] = dict(
            coarse_steps=horizon, errors=err,
            note="FP32 storage against the FP64 build of the same run (same inlet noise); "
                 "p' = cs^2 (rho - rho0)")
        del mom
        torch.cuda.empty_cache()
    return res


def serving_errors(be, lbm, torch, side=256, steps=2000):
    """Storage error of the served job kinds: the smallest jobs of the mix
    (side x side, the shortest length) in FP32 and FP16-shifted storage
    against the FP64 build of the same job (same fields, noise and step
    count; the parity tests match served FP64 jobs to the oracle within
    1e-12): relative L2 error of p' = cs^2 (rho - rho0) and of u."""
    out = {}
    for kind in ("cylinder", "pulse"):
        res = {}
        for st in ("f64", "f32", "f16s"):
            job = dict(id=0, kind=kind, nx=side, ny=side, ma=0.2, steps=steps, seed=7,
                       storage=st, arrival=0.0)
            h = be.start(job)
            lbm.lbm_step(h["ctx"], steps)
            rho = torch.empty(side * side, dtype=torch.float64, device="cuda")
            u = torch.empty(3, side * side, dtype=torch.float64, device="cuda")
            lbm.lbm_moments(h["ctx"], 0, rho, u)
            be.finish(h)
            res[st] = (rho, u)
        r64, u64 = res["f64"]
        live = r64 != 0
        p64 = (r64 - 1.0)[live]
        out[kind] = {st: dict(p_rel_l2=float((res[st][0] - r64)[live].norm() / p64.norm()),
                              u_rel_l2=float((res[st][1] - u64)[:, live].norm()
                                             / u64[:, live].norm()),
                              rho_max_abs=float((res[st][0] - r64)[live].abs().max()))
                     for st in ("f32", "f16s")}
    out["job"] = "%d x %d, Ma 0.2, %d steps" % (side, side, steps)
    out["note"] = ("p' relative L2 is over the whole p' field; in the periodic pulse job the "
                   "1e-3 pulse has spread over the box after 2000 steps, so p' is small and its "
                   "relative error large; rho_max_abs is the largest density error, to be read "
                   "against the initial pulse amplitude 1e-3")
    return out


def serving_bench(n_jobs, step_scale, loads, budget_gib, quantum):
    """Continuous-batching serving of the D2Q9 job mix: first all jobs at
    t = 0 (saturated throughput), then a seeded Poisson stream offered at
    each of `loads` times that throughput; p50/p99 latency from arrival to
    result."""
    from paper_1710_02065_amd import serve
    from paper_1710_02065_amd import workloads as W
    be = serve.GpuBackend()
    budget = int(budget_gib * 2 ** 30)
    warm = W.serving_jobs(4, 99, 1e9, side_range=(128, 256), step_range=(40, 80))
    serve.Server(be, budget, quantum).run(warm)
    sat_jobs = W.serving_jobs(n_jobs, 5, 1e9, step_scale=step_scale)
    sat = serve.Server(be, budget, quantum).run(sat_jobs).summary()
    work = sum(j["nx"] * j["ny"] * j["steps"] for j in sat_jobs) / len(sat_jobs)
    per_load = {}
    for load in loads:
        rate = load * sat["mlups"] * 1e6 / work
        jobs = W.serving_jobs(n_jobs, 5, rate, step_scale=step_scale)
        st = serve.Server(be, budget, quantum).run(jobs).summary()
        per_load["%.2f" % load] = dict(
            arrival_rate_per_s=round(rate, 3), p50_latency_s=round(st["p50_latency_s"], 4),
            p99_latency_s=round(st["p99_latency_s"], 4), p50_queue_s=round(st["p50_queue_s"], 4),
            p99_queue_s=round(st["p99_queue_s"], 4), mlups=round(st["mlups"], 1),
            peak_resident_gib=round(st["peak_bytes"] / 2 ** 30, 3))
    errors = serving_errors(be, be.lbm, be.torch)
    return dict(
        storage_error_vs_f64=errors,
        workload="D2Q9 job mix: half cylinder channels, half acoustic pulses, sides U{256..2048}, "
                 "Ma U[0.05, 0.3], steps U{2000..20000} x %g, half FP32 / half FP16-shifted "
                 "storage, Poisson arrivals (seed 5)" % step_scale,
        jobs=n_jobs, saturated_mlups=round(sat["mlups"], 1),
        saturated_p50_latency_s=round(sat["p50_latency_s"], 4),
        saturated_p99_latency_s=round(sat["p99_latency_s"], 4),
        budget_gib=budget_gib, quantum_steps=quantum, offered_load=per_load)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--block", type=int, default=-1,
                    help="workgroup size of the headline sweep (-1: the fixed HEADLINE_BLOCK "
                         "for FP32, the autotuner for M32; 0: the autotuner)")
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of --steps steps each; the median is reported")
    ap.add_argument("--storage", default="f32", choices=["f32", "m32"],
                    help="storage of the timed headline run: FP32 populations, or the "
                         "FP32 moment storage (10 values per cell)")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="whole-grid oracle steps of the CPU leg (about 20 s on 16 cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-sharding", action="store_true")
    ap.add_argument("--config-steps", type=int, default=500)
    ap.add_argument("--configs", default="c1,c2,cylinder_levels,stability,c4",
                    help="comma-separated subset of the other configurations to run")
    ap.add_argument("--shedding-steps", type=int, default=160000,
                    help="cylinder channel steps for C_L / St (0: skip)")
    ap.add_argument("--precision-horizons", type=lambda s: [int(x) for x in s.split(",")],
                    default=[50, 100, 200, 500, 1000, 2000, 5000])
    ap.add_argument("--serve-jobs", type=int, default=160)
    ap.add_argument("--serve-step-scale", type=float, default=1.0)
    ap.add_argument("--serve-loads", type=lambda s: [float(x) for x in s.split(",")],
                    default=[0.5, 0.8])
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-quantum", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 2 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU only; --gpus %d is not supported "
              "(the z-slab decomposition is timed on one GPU under \"sharding\")"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1710_02065_amd import lbm
    from paper_1710_02065_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n = args.n
    N = n ** 3
    U = 0.1 / math.sqrt(3)
    log("generating fields %d^3" % n)
    rho_np, u_np = W.taylor_green_3d(n, U, pulse_amp=1e-3, pulse_sigma=8.0)
    dev = torch.device("cuda", 0)
    fields = (torch.from_numpy(rho_np).to(dev), torch.from_numpy(u_np).to(dev))
    del rho_np, u_np

    if args.copy_calibration:
        a = torch.empty(2 ** 31 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    copy_gbs = copy_bandwidth(torch)
    hs = args.storage
    moment = hs == "m32"
    log("timing %s: %d warmup + %d steps" % (hs, args.warmup, args.steps))
    block = args.block if args.block >= 0 else (0 if moment else HEADLINE_BLOCK)
    sim32, ms32, windows = run_gpu(lbm, torch, hs, n, args.steps, args.warmup, fields, block,
                                   windows=args.windows)
    mlups32 = N * args.steps / (ms32 * 1e3)
    bytes_lup = 2 * (10 if moment else 19) * 4
    per_launch_s = ms32 / 1e3 / args.steps
    wg32 = sim32.block
    achieved = bytes_lup * N / per_launch_s / 1e9
    kname = "k_msweep_d3q19_m32_256" if moment else "k_sweep_d3q19_f32_256"
    traffic = measured_traffic(kname) if n == 256 else None

    variants = {}
    precision = {}
    del sim32
    torch.cuda.empty_cache()
    if not args.no_variants:
        for st in [v for v in ("f32", "f16s", "f32s", "f64", "m32", "m64") if v != hs]:
            log("timing %s" % st)
            sv, msv, _ = run_gpu(lbm, torch, st, n, args.steps, args.warmup, fields,
                                 HEADLINE_BLOCK if st == "f32" else 0)
            # the moment storages move 10 values per cell each way, not 19
            vals = 10 if st.startswith("m") else 19
            b = 2 * vals * lbm.STORAGE_BYTES[lbm.STORAGE[st]]
            mv = N * args.steps / (msv * 1e3)
            variants[st] = dict(value=round(mv, 1), unit="MLUPS", bytes_per_lup=b,
                                hbm_gbs=round(b * N / (msv / 1e3 / args.steps) / 1e9, 1),
                                speedup_vs_headline=round(mv / mlups32, 3), workgroup=sv.block)
            if st.startswith("m"):
                variants[st]["planes_per_workgroup"] = sv.block // 16
            del sv
            torch.cuda.empty_cache()
        # regularization order on D3Q27 (the lattice that resolves up to sixth
        # order): third order against the full recursive expansion
        order = {}
        for st in ("f32", "f16s", "m32"):
            for name, fl in (("third", 0), ("full", lbm.LBM_FULL_ORDER)):
                log("timing d3q27 %s %s" % (st, name))
                sv, msv, _ = run_gpu(lbm, torch, st, n, max(args.steps // 4, 50),
                                     args.warmup // 4, fields, 0, lattice=27, flags=fl)
                b = 2 * (10 if st.startswith("m") else 27) * lbm.STORAGE_BYTES[lbm.STORAGE[st]]
                ns = max(args.steps // 4, 50)
                order["d3q27_%s_%s" % (st, name)] = dict(
                    mlups=round(N * ns / (msv * 1e3), 1), bytes_per_lup=b,
                    hbm_gbs=round(b * N * ns / (msv / 1e3) / 1e9, 1), workgroup=sv.block)
                del sv
                torch.cuda.empty_cache()
        variants["regularization_order_d3q27_%d" % n] = order
        log("precision study: f64 / f32 / f32s / f16s side by side")
        precision = precision_study(lbm, torch, n, fields, args.precision_horizons)

    out = {
        "metric": METRIC,
        "value": round(mlups32, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32 / args.steps, 5),
        "timing": "median of %d windows of %d steps (HIP events on the launch stream); "
                  "every window in ms: %s" % (len(windows), args.steps,
                                             ", ".join("%.4f" % w for w in windows)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "D3Q19 %d^3 periodic, Taylor-Green U=0.1cs + Gaussian pulse 1e-3 "
                        "sigma 8, tau 0.52, %s (fused pull + rrBGK sweep)"
                        % (n, "FP32 moment storage" if moment else "FP32 storage"),
            "lattice": "D3Q19", "cells": N, "storage": hs, "tau": 0.52,
            "parallelism": "single GPU"},
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_lup * N,
            "measured_copy_gbs": copy_gbs,
            "kernel": "k_msweep<D3Q19, float>" if moment else "k_sweep<D3Q19, f32>"},
    }
    if variants:
        out["variants"] = variants
    if precision:
        out["precision_vs_f64_build"] = precision
        if "f16s" in variants:
            meets = [int(T) for T, row in precision.items() if row["f16s"]["p_rel_l2"] <= 1e-3]
            out["f16s_speedup_at_1e-3"] = {
                "speedup_vs_f32": variants["f16s"]["speedup_vs_headline"],
                "horizons_within_1e-3": meets,
                "note": "FP16-shifted storage over FP32 on the same GPU; the horizons (steps) "
                     "at which its acoustic-pressure error against the FP64 build is at most "
                     "1e-3 relative (none: it meets the bar at no horizon measured)"}
    out["config"]["workgroup"] = wg32
    if not args.no_sharding and n % 8 == 0:
        log("slab decomposition rehearsal (8 z-slabs)")
        out["sharding"] = slab_rehearsal(lbm, torch, n, fields, min(args.steps, 500), mlups32)
    if not args.no_configs:
        log("other configurations")
        out["configs"] = other_configs(lbm, torch, args.config_steps, args.shedding_steps,
                                       which=tuple(args.configs.split(",")))
        torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving: %d jobs, step scale %g" % (args.serve_jobs, args.serve_step_scale))
        out["serving"] = serving_bench(args.serve_jobs, args.serve_step_scale, args.serve_loads,
                                       args.serve_budget_gib, args.serve_quantum)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        anchors = None
        if not args.no_variants:
            log("anchor runs: %d steps in each storage" % args.cpu_steps)
            anchors = anchor_states(lbm, torch, n, fields, args.cpu_steps)
        del fields
        torch.cuda.empty_cache()
        log("cpu baseline (oracle): %d steps" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_steps, anchors)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
