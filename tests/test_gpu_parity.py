"""GPU (HIP, gfx950) against the FP64 oracle, through the C ABI.

Bars: FP64 build within 1e-12 normwise (max |gpu - oracle| / max |oracle|)
on every case; FP32 formats within 2e-6 and the FP16-shifted format within
2e-4 of one oracle step taken from the GPU's own stored state (the error
of one step's arithmetic plus one storage rounding, derived in the design
notes); integer-valued results (step counters, masks, bitwise replays)
exactly.
"""
import math

import numpy as np
import pytest

from paper_1710_02065_amd import workloads as W
import oracle as O
from tests.pair import gpu_sim, log, normwise, oracle_grid, run_both

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
TOL = {"f32": 2e-6, "f32s": 2e-6, "f16s": 2e-4}


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dim(q):
    return 2 if q == 9 else 3


RAGGED = {9: (45, 37, 1), 19: (17, 13, 11), 27: (15, 12, 9)}


@pytest.mark.parametrize("q", [9, 19, 27])
def test_init_parity_f64(q):
    shape = RAGGED[q]
    rho, u, p = W.random_state(shape, seed=10 + q, d=dim(q))
    case = dict(name="init", q=q, shape=shape, tau=0.57)
    gf, of, _, _ = run_both(case, 0, "f64", rho, u, p)
    assert normwise(gf, of) <= F64_TOL


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("steps", [1, 7])
def test_periodic_step_parity_f64(q, steps):
    shape = RAGGED[q]
    rho, u, p = W.random_state(shape, seed=20 + q, d=dim(q))
    case = dict(name="periodic", q=q, shape=shape, tau=0.53)
    gf, of, _, _ = run_both(case, steps, "f64", rho, u, p)
    assert normwise(gf, of) <= F64_TOL


@pytest.mark.parametrize("q,shape", [(9, (1, 1, 1)), (9, (1, 5, 1)), (9, (7, 1, 1)),
                                     (19, (1, 1, 1)), (19, (2, 3, 1)), (27, (3, 1, 2))])
def test_degenerate_shapes_f64(q, shape):
    rho, u, p = W.random_state(shape, seed=30, d=dim(q))
    case = dict(name="degenerate", q=q, shape=shape, tau=0.8)
    gf, of, _, _ = run_both(case, 3, "f64", rho, u, p)
    assert normwise(gf, of) <= F64_TOL


def channel_case(q):
    """Cylinder-in-channel stand-in: inlet column with noise, free-slip
    sides, zero-gradient outflow, sponge on the outflow face, SOLID disc."""
    if q == 9:
        nx, ny, nz = 96, 48, 1
        mask = W.cylinder_mask(nx, ny, 12, 30, 24)
        fb = (2, 2, 1, 1, 0, 0)
        sw = (0, 16, 0, 0, 0, 0)
    else:
        nx, ny, nz = 40, 18, 14
        mask = W.cylinder_mask(nx, ny, 6, 12, 9)
        mask = np.tile(mask, nz)
        fb = (2, 2, 1, 1, 2, 2)
        sw = (0, 10, 0, 0, 4, 4)
    return dict(name="channel", q=q, shape=(nx, ny, nz), tau=0.56, ma=0.2, u_dir=(1, 0, 0),
                face_bc=fb, sponge_width=sw, chi_max=0.3, rho_ref=1.0,
                u_ref=(0.2 / math.sqrt(3), 0, 0), seed=5, inlet_noise=0.02, mask=mask)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_boundary_rules_parity_f64(q):
    case = channel_case(q)
    shape = case["shape"]
    U = case["ma"] / math.sqrt(3)
    rho, u = W.uniform_perturbed(shape, U, (1, 0, 0), seed=3, rel_noise=1e-2, d=dim(q))
    gf, of, sim, g = run_both(case, 25, "f64", rho, u)
    assert normwise(gf, of) <= F64_TOL
    r_g, u_g = sim.moments()
    r_o, u_o = g.moments()
    assert normwise(r_g.cpu().numpy(), r_o) <= F64_TOL
    assert normwise(u_g.cpu().numpy(), u_o) <= F64_TOL


def test_closed_box_and_jet_inlet_parity_f64():
    shape = (20, 18, 16)
    mask = W.closed_box_mask(*shape)
    mask[W.jet_inlet_mask(*shape, D=6) == W.INLET] = W.INLET
    rho, u, p = W.random_state(shape, seed=4, d=3, u_amp=0.02)
    case = dict(name="box+jet", q=27, shape=shape, tau=0.51, ma=0.3, seed=11,
                inlet_noise=0.02, mask=mask, face_bc=(2, 2, 1, 1, 2, 2),
                sponge_width=(0, 6, 3, 3, 3, 3), chi_max=0.2)
    gf, of, _, _ = run_both(case, 15, "f64", rho, u, p)
    assert normwise(gf, of) <= F64_TOL


def test_taylor_green_config_f64():
    """D2Q9 128^2 periodic, FP64, tau 0.6, U = 0.05, 1000 steps."""
    n, U = 128, 0.05
    rho, u, _ = W.taylor_green_2d(n, U)
    case = dict(name="tg128", q=9, shape=(n, n, 1), tau=0.6)
    gf, of, sim, g = run_both(case, 1000, "f64", rho, u)
    assert normwise(gf, of) <= F64_TOL
    r_g, u_g = sim.moments()
    r_o, u_o = g.moments()
    assert normwise(u_g.cpu().numpy(), u_o) <= F64_TOL
    assert sim.time == 1000


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("storage", ["f32", "f32s", "f16s"])
def test_low_precision_single_step(q, storage):
    """One step in FP32 arithmetic from the GPU's stored state against one
    oracle step from the same (exactly converted) state."""
    shape = RAGGED[q]
    rho, u, p = W.random_state(shape, seed=40 + q, d=dim(q))
    case = channel_case(q) if q == 19 else dict(name="lowprec", q=q, shape=shape, tau=0.52)
    if q == 19:
        shape = case["shape"]
        rho, u, p = W.random_state(shape, seed=40 + q, d=3)
    log("lowprec q=%d storage=%s" % (q, storage))
    sim = gpu_sim(case, storage)
    sim.init(rho, u, p, case.get("mask"))
    sim.step(2)
    f0 = sim.populations().cpu().numpy()
    sim.step(1)
    f1 = sim.populations().cpu().numpy()
    sim.sync()
    g = oracle_grid(case)
    g.set_populations(f0)
    g.t = 2
    g.step(1)
    assert normwise(f1, g.f) <= TOL[storage]


def test_moments_and_probe_match_oracle():
    case = channel_case(9)
    rho, u = W.uniform_perturbed(case["shape"], 0.1, (1, 0, 0), seed=8, rel_noise=0.05, d=2)
    _, _, sim, g = run_both(case, 10, "f64", rho, u)
    r_o, _ = g.moments()
    cells = np.array([0, 5, 100, 2000, 4607], dtype=np.int64)
    pr = sim.probe(cells).cpu().numpy()
    np.testing.assert_allclose(pr, r_o[cells], rtol=1e-13, atol=0)


def test_checkpoint_resume_bitwise():
    case = dict(name="resume", q=19, shape=(20, 16, 12), tau=0.55, face_bc=(2, 2, 1, 1, 0, 0),
                sponge_width=(0, 5, 0, 0, 0, 0), chi_max=0.3)
    rho, u, p = W.random_state(case["shape"], seed=9, d=3)
    for storage in ("f32", "f16s", "f64"):
        log("resume storage=%s" % storage)
        a = gpu_sim(case, storage).init(rho, u, p).step(20)
        fa = a.populations().cpu().numpy()
        b = gpu_sim(case, storage).init(rho, u, p).step(10)
        fb = b.populations()
        c = gpu_sim(case, storage).init(rho, u, p)
        c.set_populations(fb)
        c.step(10)
        fc = c.populations().cpu().numpy()
        np.testing.assert_array_equal(fa, fc)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_checkpoint_resume_with_inlet_noise_bitwise(storage):
    """Inlet noise depends on the time index: a run resumed into a fresh
    context (initialised with other fields, then populations and time
    restored) continues bitwise like the uninterrupted run."""
    case = channel_case(9)
    rho, u = W.uniform_perturbed(case["shape"], 0.1, (1, 0, 0), seed=8, rel_noise=0.05, d=2)
    log("resume with noise storage=%s" % storage)
    a = gpu_sim(case, storage).init(rho, u, None, case["mask"]).step(30)
    b = gpu_sim(case, storage).init(rho, u, None, case["mask"]).step(13)
    ck = b.checkpoint()
    c = gpu_sim(case, storage).init(None, None, None, case["mask"]).restore(ck)
    assert c.time == 13
    c.step(17)
    np.testing.assert_array_equal(c.populations().cpu().numpy(), a.populations().cpu().numpy())
    # without the time the noise differs
    d = gpu_sim(case, storage).init(None, None, None, case["mask"])
    d.set_populations(ck["pops"][0])
    d.step(17)
    assert not np.array_equal(d.populations().cpu().numpy(), a.populations().cpu().numpy())


def test_run_to_run_bitwise_deterministic():
    case = channel_case(9)
    rho, u = W.uniform_perturbed(case["shape"], 0.1, (1, 0, 0), seed=8, rel_noise=0.05, d=2)
    outs = []
    for _ in range(2):
        s = gpu_sim(case, "f32").init(rho, u, None, case["mask"]).step(50)
        outs.append(s.populations().cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_graph_replay_matches_eager(storage):
    from paper_1710_02065_amd import lbm
    case = dict(name="graph", q=19, shape=(24, 20, 16), tau=0.55)
    rho, u, p = W.random_state(case["shape"], seed=12, d=3)
    log("graph storage=%s" % storage)
    a = gpu_sim(case, storage).init(rho, u, p)
    b = gpu_sim(case, storage, flags=lbm.LBM_NO_GRAPH).init(rho, u, p)
    for n in (200, 70, 64, 3, 130):
        a.step(n)
        b.step(n)
        fa = a.populations().cpu().numpy()
        fb = b.populations().cpu().numpy()
        np.testing.assert_array_equal(fa, fb)
    assert a.time == b.time == 467


@pytest.mark.parametrize("bad", ["negative", "nan"])
def test_watchdog_reports_instability(bad):
    """A cell whose pulled density is non-positive or not finite sets the
    sticky flag; the next sync reports LBM_EUNSTABLE.  (A mildly negative
    initial density is smoothed by streaming: the pulled density of that
    cell is 1 - 4/9 * 1.5 > 0, so the forcing is strong.)"""
    from paper_1710_02065_amd import lbm
    case = dict(name="unstable-" + bad, q=9, shape=(16, 16, 1), tau=0.6)
    rho = np.ones(256)
    u = np.zeros((3, 256))
    if bad == "negative":
        rho[37] = -100.0
    else:
        u[0, 37] = np.nan
    s = gpu_sim(case, "f32").init(rho, u)
    s.sync()
    s.step(2)
    with pytest.raises(lbm.LbmError) as e:
        s.sync()
    assert e.value.code == lbm.LBM_EUNSTABLE
    with pytest.raises(lbm.LbmError):  # sticky
        s.sync()


def test_step_batch_equals_solo():
    from paper_1710_02065_amd import lbm
    cases = [dict(name="b0", q=9, shape=(64, 48, 1), tau=0.6),
             dict(name="b1", q=9, shape=(37, 91, 1), tau=0.7, face_bc=(2, 2, 1, 1, 0, 0),
                  sponge_width=(0, 8, 0, 0, 0, 0), chi_max=0.2),
             dict(name="b2", q=9, shape=(128, 30, 1), tau=0.52)]
    steps = [40, 13, 77]
    fields = [W.random_state(c["shape"], seed=50 + k, d=2) for k, c in enumerate(cases)]
    for storage in ("f32", "f16s"):
        log("batch storage=%s" % storage)
        solo = []
        for c, f, n in zip(cases, fields, steps):
            solo.append(gpu_sim(c, storage).init(*f).step(n).populations().cpu().numpy())
        sims = [gpu_sim(c, storage).init(*f) for c, f in zip(cases, fields)]
        lbm.lbm_step_batch([s.ctx for s in sims], steps)
        for s, ref, n in zip(sims, solo, steps):
            np.testing.assert_array_equal(s.populations().cpu().numpy(), ref)
            assert s.time == n


def test_step_batch_concurrent_groups_equal_solo():
    """Eight groups in one batched call (FP32 / F16S storage x periodic /
    general path x workgroup 128 / 256): the first runs on the contexts'
    stream, the other seven on streams of the library's own, joined back
    before the populations are read on the contexts' stream without a
    host synchronisation.  Two calls in a row (the second reuses the
    streams and the captured graphs), step counts with graph replays,
    tails and an idle job, a large job beside small ones: every context
    bitwise equal to stepping it alone."""
    from paper_1710_02065_amd import lbm
    periodic = dict(q=9, tau=0.6)
    general = dict(q=9, tau=0.7, face_bc=(2, 2, 1, 1, 0, 0), sponge_width=(0, 8, 0, 0, 0, 0),
                   chi_max=0.2)
    cases, blocks = [], []
    for storage in ("f32", "f16s"):
        for kind, base in (("periodic", periodic), ("general", general)):
            for block in (128, 256):
                shape = (512, 384, 1) if (storage, kind, block) == ("f32", "general", 128) \
                    else (48 + 8 * len(cases), 37, 1)
                cases.append(dict(base, name="%s-%s-%d" % (storage, kind, block), shape=shape,
                                  storage=storage))
                blocks.append(block)
    first = [40, 13, 77, 0, 33, 16, 5, 21]
    second = [17, 32, 3, 18, 0, 48, 29, 7]
    fields = [W.random_state(c["shape"], seed=90 + k, d=2) for k, c in enumerate(cases)]
    solo = []
    for c, f, b, n1, n2 in zip(cases, fields, blocks, first, second):
        log("batch lanes solo %s" % c["name"])
        solo.append(gpu_sim(c, c["storage"], block=b).init(*f).step(n1 + n2)
                    .populations().cpu().numpy())
    sims = [gpu_sim(c, c["storage"], block=b).init(*f) for c, f, b in zip(cases, fields, blocks)]
    log("batch lanes: two batched calls over eight groups")
    lbm.lbm_step_batch([s.ctx for s in sims], first)
    lbm.lbm_step_batch([s.ctx for s in sims], second)
    got = [s.populations() for s in sims]  # queued on the contexts' stream
    for s, g, ref, c, n1, n2 in zip(sims, got, solo, cases, first, second):
        np.testing.assert_array_equal(g.cpu().numpy(), ref, err_msg=c["name"])
        assert s.time == n1 + n2


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_full_size_d3q19_sampled_parity(storage):
    """D3Q19 256^3 periodic, Taylor-Green + acoustic pulse, in the launch
    configuration the benchmark times.  After two GPU steps, a 24^3 block
    (plus its one-cell halo) of the stored state is stepped once by the
    oracle and compared with the GPU's third step on the block interior."""
    n = 256
    U = 0.1 / math.sqrt(3)
    rho, u = W.taylor_green_3d(n, U, pulse_amp=1e-3, pulse_sigma=8.0)
    case = dict(name="c3", q=19, shape=(n, n, n), tau=0.52)
    log("full-size D3Q19 256^3 storage=%s" % storage)
    sim = gpu_sim(case, storage).init(rho, u)
    del rho, u
    sim.step(2)
    f0 = sim.populations()
    lo = np.array([100, 117, 30])  # block origin (x, y, z) incl. halo
    B = 26
    idx = ((np.arange(lo[2], lo[2] + B)[:, None, None] * n
            + np.arange(lo[1], lo[1] + B)[None, :, None]) * n
           + np.arange(lo[0], lo[0] + B)[None, None, :]).ravel()
    tidx = torch.from_numpy(idx).to(f0.device)
    blk0 = f0[:, tidx].cpu().numpy()
    del f0
    sim.step(1)
    f1 = sim.populations()
    blk1 = f1[:, tidx].cpu().numpy()
    del f1
    sim.sync()
    g = oracle_grid(dict(q=19, shape=(B, B, B), tau=0.52))
    g.set_populations(blk0)
    g.step(1)
    inner = np.zeros((B, B, B), dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    inner = inner.ravel()
    assert normwise(blk1[:, inner], g.f[:, inner]) <= TOL[storage]


def test_full_size_channel_one_step():
    """D2Q9 2048x1024 cylinder channel (D = 100 at (400, 512), inlet column,
    free-slip sides, outflow with a 128-column sponge), FP32: one oracle
    step from the GPU's stored state over the whole grid."""
    nx, ny, D = 2048, 1024, 100
    U = 0.2 / math.sqrt(3)
    tau = 0.5 + 3 * U * D / 150
    mask = W.cylinder_mask(nx, ny, D, 400, 512)
    case = dict(name="c2", q=9, shape=(nx, ny, 1), tau=tau, ma=0.2, face_bc=(2, 2, 1, 1, 0, 0),
                sponge_width=(0, 128, 0, 0, 0, 0), chi_max=0.2, rho_ref=1.0,
                u_ref=(U, 0, 0), seed=2, mask=mask)
    rho, u = W.uniform_perturbed((nx, ny, 1), U, (1, 0, 0), seed=2, rel_noise=1e-4, d=2)
    log("full-size D2Q9 2048x1024 channel f32")
    sim = gpu_sim(case, "f32").init(rho, u, None, mask)
    sim.step(5)
    f0 = sim.populations().cpu().numpy()
    sim.step(1)
    f1 = sim.populations().cpu().numpy()
    sim.sync()
    g = oracle_grid(case)
    g.set_populations(f0)
    g.t = 5
    g.step(1)
    assert normwise(f1, g.f) <= TOL["f32"]


def test_autotune_keeps_state_and_caches(tmp_path, monkeypatch):
    from paper_1710_02065_amd import lbm
    monkeypatch.setenv("HRLBM_TUNE_CACHE", str(tmp_path / "tune.json"))
    case = dict(name="tune", q=19, shape=(48, 40, 36), tau=0.55)
    rho, u, p = W.random_state(case["shape"], seed=13, d=3)
    log("autotune")
    a = gpu_sim(case, "f32").init(rho, u, p).step(3)
    f0 = a.populations().cpu().numpy()
    best = lbm.lbm_autotune(a.ctx, 1)
    assert best in (64, 128, 256, 512, 1024)
    np.testing.assert_array_equal(a.populations().cpu().numpy(), f0)
    a.step(4)
    b = gpu_sim(case, "f32", block=64).init(rho, u, p).step(7)
    np.testing.assert_array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    text = (tmp_path / "tune.json").read_text()
    assert ": %d" % best in text
    c = gpu_sim(case, "f32").init(rho, u, p)  # picks the cached size
    c.step(7)
    np.testing.assert_array_equal(c.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_poisoned_job_does_not_change_the_others():
    """A batch where one context goes unstable: it reports LBM_EUNSTABLE,
    the others report OK and match their solo runs bitwise."""
    from paper_1710_02065_amd import lbm
    cases = [dict(name="ok0", q=9, shape=(64, 48, 1), tau=0.6),
             dict(name="bad", q=9, shape=(40, 40, 1), tau=0.6),
             dict(name="ok1", q=9, shape=(50, 70, 1), tau=0.7)]
    fields = [W.random_state(c["shape"], seed=70 + k, d=2) for k, c in enumerate(cases)]
    rho_bad = fields[1][0].copy()
    rho_bad[100] = np.nan
    fields[1] = (rho_bad,) + fields[1][1:]
    log("poisoned batch")
    solo = [gpu_sim(c, "f32").init(*f).step(30).populations().cpu().numpy()
            for c, f in zip(cases, fields)]
    sims = [gpu_sim(c, "f32").init(*f) for c, f in zip(cases, fields)]
    lbm.lbm_step_batch([s.ctx for s in sims], [30, 30, 30])
    for k in (0, 2):
        np.testing.assert_array_equal(sims[k].populations().cpu().numpy(), solo[k])
        sims[k].sync()
    with pytest.raises(lbm.LbmError) as e:
        sims[1].sync()
    assert e.value.code == lbm.LBM_EUNSTABLE


def _force_cases():
    box = (20, 18, 16)
    mask = W.closed_box_mask(*box)
    mask[W.jet_inlet_mask(*box, D=6) == W.INLET] = W.INLET
    boxcase = dict(name="box+jet", q=19, shape=box, tau=0.55, ma=0.2, seed=3,
                   inlet_noise=0.01, mask=mask, face_bc=(2, 2, 1, 1, 2, 2),
                   sponge_width=(0, 6, 3, 3, 3, 3), chi_max=0.2)
    return [channel_case(9), channel_case(19), channel_case(27), boxcase]


@pytest.mark.parametrize("k", range(4))
def test_force_parity_f64(k):
    """Momentum-exchange force on the SOLID cells against the oracle's,
    normwise within 1e-12, at two time levels; repeated calls bitwise."""
    case = _force_cases()[k]
    shape = case["shape"]
    d = dim(case["q"])
    rho, u = W.uniform_perturbed(shape, 0.1, (1, 0, 0), seed=9, rel_noise=1e-2, d=d)
    sim = gpu_sim(case, "f64")
    log("force %s q=%d" % (case["name"], case["q"]))
    sim.init(rho, u, None, case["mask"])
    g = oracle_grid(case).init(rho, u)
    for steps in (0, 17):
        sim.step(steps)
        g.step(steps)
        F1 = sim.force().cpu().numpy()
        F2 = sim.force().cpu().numpy()
        sim.sync()
        Fo = g.force()
        assert np.abs(Fo).max() > 1e-3
        assert normwise(F1, Fo) <= F64_TOL
        assert np.array_equal(F1, F2)


@pytest.mark.parametrize("storage", ["f32", "f32s", "f16s"])
def test_force_low_precision_same_state(storage):
    """In the narrow formats the force is summed in FP64 from the stored
    values: the oracle's force of the same (exactly converted) state agrees
    up to summation order."""
    case = channel_case(19)
    rho, u = W.uniform_perturbed(case["shape"], 0.1, (1, 0, 0), seed=2, rel_noise=1e-2, d=3)
    sim = gpu_sim(case, storage)
    log("force lowprec %s" % storage)
    sim.init(rho, u, None, case["mask"])
    sim.step(9)
    F = sim.force().cpu().numpy()
    f = sim.populations().cpu().numpy()
    sim.sync()
    g = oracle_grid(case)
    g.set_populations(f)
    assert normwise(F, g.force()) <= 1e-13


def test_force_series_into_slices_and_no_mask_is_zero():
    case = channel_case(9)
    rho, u = W.uniform_perturbed(case["shape"], 0.1, (1, 0, 0), seed=4, rel_noise=1e-2, d=2)
    sim = gpu_sim(case, "f32")
    log("force series")
    sim.init(rho, u, None, case["mask"])
    series = torch.zeros(5, 3, dtype=torch.float64, device="cuda")
    for k in range(5):
        sim.step(3)
        sim.force(out=series[k])
    ref = sim.force().cpu().numpy()
    sim.sync()
    assert np.array_equal(series[4].cpu().numpy(), ref)
    assert np.all(series[:, 0].cpu().numpy() != 0)
    plain = gpu_sim(dict(q=9, shape=(32, 16, 1)), "f32")
    plain.init()
    assert np.all(plain.force().cpu().numpy() == 0.0)


def test_accumulate_matches_oracle_moments():
    """Running sums of rho - rho0 and its square over sampled steps against
    the same sums of the oracle's densities.  The oracle forms rho - rho0
    from a full rho of about 1, so each term carries an absolute rounding of
    about 1e-16 against deviations of about 1e-3: bound 1e-11 normwise."""
    case = channel_case(9)
    rho, u = W.uniform_perturbed(case["shape"], 0.1, (1, 0, 0), seed=12, rel_noise=2e-2, d=2)
    sim = gpu_sim(case, "f64")
    log("accumulate")
    sim.init(rho, u, None, case["mask"])
    g = oracle_grid(case).init(rho, u)
    N = int(np.prod(case["shape"]))
    s1 = torch.zeros(N, dtype=torch.float64, device="cuda")
    s2 = torch.zeros(N, dtype=torch.float64, device="cuda")
    o1, o2 = np.zeros(N), np.zeros(N)
    fluid = case["mask"] != W.SOLID
    for k in range(6):
        sim.step(4)
        g.step(4)
        sim.accumulate(s1, s2)
        x = np.where(fluid, g.moments()[0] - 1.0, 0.0)
        o1 += x
        o2 += x * x
    sim.sync()
    assert np.abs(o1).max() > 1e-4
    assert normwise(s1.cpu().numpy(), o1) <= 1e-11
    assert normwise(s2.cpu().numpy(), o2) <= 1e-11
    assert np.all(s1.cpu().numpy()[~fluid] == 0.0)


def test_totals_match_oracle_and_are_conserved():
    """Global mass (relative to rest) and momentum against the oracle's sums
    in FP64; in a periodic run they stay constant (FP64: to rounding; FP32:
    within the storage rounding of the deviations)."""
    case = channel_case(19)
    rho, u = W.uniform_perturbed(case["shape"], 0.1, (1, 0, 0), seed=13, rel_noise=2e-2, d=3)
    sim = gpu_sim(case, "f64")
    log("totals channel")
    sim.init(rho, u, None, case["mask"])
    g = oracle_grid(case).init(rho, u)
    sim.step(11)
    g.step(11)
    T = sim.totals().cpu().numpy()
    sim.sync()
    xi, _, _ = O.lattice(19)
    upd = case["mask"] != W.SOLID
    want = np.concatenate([[g.f[:, upd].sum() - upd.sum() * 1.0],
                           (g.f[:, upd].sum(axis=1)[:, None] * xi).sum(axis=0)])
    scale = np.abs(g.f[:, upd]).sum()
    np.testing.assert_allclose(T, want, rtol=0, atol=64 * np.finfo(float).eps * scale)
    for storage, tol in (("f64", 1e-13), ("f32", 1e-6)):
        shape = RAGGED[27]
        rho, u, p = W.random_state(shape, seed=14, d=3, u_amp=0.05)
        s = gpu_sim(dict(q=27, shape=shape, tau=0.6), storage)
        log("totals periodic %s" % storage)
        s.init(rho, u, p)
        t0 = s.totals().cpu().numpy()
        s.step(50)
        t1 = s.totals().cpu().numpy()
        s.sync()
        N = np.prod(shape)
        assert np.abs(t1 - t0).max() <= tol * N


def _circular_case(q):
    if q == 9:
        shape = (64, 48, 1)
        center = (31.5, 23.5, 0.0)
        r0, r1 = 14.0, 40.0
    else:
        shape = (28, 24, 20)
        center = (13.5, 11.5, 9.5)
        r0, r1 = 6.0, 20.0
    return shape, O.circular_sponge(shape, center, r0, r1, 0.3)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_field_sponge_parity_f64(q):
    """Circular absorbing layer with a spatially varying reference (a
    Gaussian jet-like velocity profile and a density ramp) against the
    oracle's per-cell layer, FP64 within 1e-12."""
    shape, chi = _circular_case(q)
    d = dim(q)
    N = int(np.prod(shape))
    x = np.arange(N) % shape[0]
    y = (np.arange(N) // shape[0]) % shape[1]
    rho_ref = 1.0 + 2e-3 * x / shape[0]
    u_ref = np.zeros((3, N))
    u_ref[0] = 0.05 * np.exp(-((y - shape[1] / 2) / 6.0) ** 2)
    rho, u, p = W.random_state(shape, seed=90 + q, d=d, u_amp=0.03)
    case = dict(name="field-sponge", q=q, shape=shape, tau=0.56)
    log("field sponge q=%d" % q)
    from paper_1710_02065_amd import lbm
    sim = gpu_sim(case, "f64", flags=lbm.LBM_SPONGE_FIELD)
    sim.init(rho, u, p)
    sim.set_sponge(chi, rho_ref, u_ref)
    sim.step(12)
    gf = sim.populations().cpu().numpy()
    sim.sync()
    g = oracle_grid(case).set_sponge(chi, rho_ref, u_ref).init(rho, u, p).step(12)
    assert normwise(gf, g.f) <= F64_TOL
    # the layer did act: a run without it differs
    g0 = oracle_grid(case).init(rho, u, p).step(12)
    assert normwise(g0.f, g.f) > 1e-6


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_field_sponge_low_precision_single_step(storage):
    shape, chi = _circular_case(19)
    rho, u, p = W.random_state(shape, seed=7, d=3)
    case = dict(name="field-sponge-lp", q=19, shape=shape, tau=0.56, rho_ref=1.01,
                u_ref=(0.03, 0.0, 0.0))
    from paper_1710_02065_amd import lbm
    log("field sponge lowprec %s" % storage)
    sim = gpu_sim(case, storage, flags=lbm.LBM_SPONGE_FIELD)
    sim.init(rho, u, p)
    sim.set_sponge(chi)
    sim.step(2)
    f0 = sim.populations().cpu().numpy()
    sim.step(1)
    f1 = sim.populations().cpu().numpy()
    sim.sync()
    g = oracle_grid(case).set_sponge(chi)
    g.set_populations(f0)
    g.t = 2
    g.step(1)
    assert normwise(f1, g.f) <= TOL[storage]


def test_field_sponge_rejected_above_stability_bound():
    from paper_1710_02065_amd import lbm
    shape = (16, 16, 1)
    case = dict(name="field-sponge-bad", q=9, shape=shape, tau=0.6)
    sim = gpu_sim(case, "f32", flags=lbm.LBM_SPONGE_FIELD)
    sim.init()
    chi = np.zeros(256)
    chi[17] = 2.5  # >= 4 tau = 2.4
    with pytest.raises(lbm.LbmError) as e:
        sim.set_sponge(chi)
    assert e.value.code == lbm.LBM_EINVAL
    plain = gpu_sim(case, "f32")
    plain.init()
    with pytest.raises(lbm.LbmError) as e:
        plain.set_sponge(np.zeros(256))
    assert e.value.code == lbm.LBM_ESTATE
