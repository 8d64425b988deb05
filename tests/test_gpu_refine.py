"""2:1 refinement on the GPU against the refined oracles (Sec. II.B), two
levels and nested chains of three and four:
coarse sweep with interface-moment record, two fine sweeps, RING fills at
t + 1/2 and t + 1, IMPORT by filtered fine moments.  FP64 build within 1e-12
normwise on both levels."""
import math

import numpy as np
import pytest

from paper_1710_02065_amd import workloads as W
from tests.pair import log, normwise, refined_pair, refined_sim

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def fine_shape(case):
    d = 2 if case["q"] == 9 else 3
    return tuple(2 * (case["hi"][a] - case["lo"][a]) + 1 if a < d else 1 for a in range(3))


def run_refined(case, steps, storage="f64", fields=None):
    cshape = case["shape"]
    fshape = fine_shape(case)
    d = 2 if case["q"] == 9 else 3
    if fields is None:
        fc = W.random_state(cshape, seed=1, d=d, u_amp=0.03, rho_amp=0.01, pi_amp=5e-4)
        ff = W.random_state(fshape, seed=2, d=d, u_amp=0.03, rho_amp=0.01, pi_amp=5e-4)
    else:
        fc, ff = fields
    log("refined %s q=%d coarse=%s fine=%s storage=%s steps=%d"
        % (case.get("name"), case["q"], cshape, fshape, storage, steps))
    sim = refined_sim(case, storage)
    sim.init(*fc, mask=case.get("mask"), level=0)
    sim.init(*ff, mask=case.get("fine_mask"), level=1)
    sim.step(steps)
    g0 = sim.populations(0).cpu().numpy()
    g1 = sim.populations(1).cpu().numpy()
    m0 = sim.moments(0)
    sim.sync()
    og = refined_pair(case)
    og.init(0, *fc)
    og.init(1, *ff)
    og.step(steps)
    return g0, g1, og, sim, m0


@pytest.mark.parametrize("q", [9, 19, 27])
def test_refined_periodic_parity_f64(q):
    if q == 9:
        case = dict(name="ref2d", q=9, shape=(48, 40, 1), lo=(12, 9, 0), hi=(30, 25, 0), tau=0.57)
    else:
        case = dict(name="ref3d", q=q, shape=(22, 20, 18), lo=(6, 5, 5), hi=(14, 13, 12), tau=0.55)
    g0, g1, og, _, _ = run_refined(case, 6)
    skip = og.crole == 2  # COVERED coarse nodes are never updated
    assert normwise(g0[:, ~skip], og.coarse.f[:, ~skip]) <= F64_TOL
    assert normwise(g1, og.fine.f) <= F64_TOL


@pytest.mark.parametrize("q", [19, 27])
def test_refined_with_open_boundaries_parity_f64(q):
    """Inlet disc with noise on x = 0, walls and sponge away from the patch,
    free-slip and outflow faces on the coarse level, patch in the middle."""
    shape = (30, 22, 22)
    mask = W.jet_inlet_mask(*shape, D=6)
    case = dict(name="ref-open", q=q, shape=shape, lo=(6, 6, 6), hi=(16, 15, 15), tau=0.52,
                ma=0.2, seed=3, inlet_noise=0.02, mask=mask, face_bc=(2, 2, 1, 1, 2, 2),
                sponge_width=(0, 8, 0, 0, 0, 4), chi_max=0.3)
    g0, g1, og, sim, m0 = run_refined(case, 8)
    skip = og.crole == 2
    assert normwise(g0[:, ~skip], og.coarse.f[:, ~skip]) <= F64_TOL
    assert normwise(g1, og.fine.f) <= F64_TOL
    r, _ = m0
    r = r.cpu().numpy()
    assert np.all(r[skip] == 0.0)  # COVERED cells report zero


def test_refined_shear_wave_f32_tracks_oracle():
    """The shear wave across the patch in FP32 storage: the GPU stays within
    1e-6 absolute (1e-3 of the wave amplitude) of the FP64 oracle after 200
    steps.  Bound: one FP32 rounding of populations up to 0.44 is 2.6e-8 per
    step; a random walk over 200 steps gives ~4e-7 in the velocity."""
    n, A, tau = 64, 1e-3, 0.6
    case = dict(name="shear", q=9, shape=(n, n, 1), lo=(8, 20, 0), hi=(40, 44, 0), tau=tau)
    k = 2 * math.pi / n
    Nc = n * n
    y = np.repeat(np.arange(n), n).astype(float)
    u = np.zeros((3, Nc))
    u[0] = A * np.sin(k * y)
    fx, fy, _ = fine_shape(case)
    yf = 20 + np.repeat(np.arange(fy), fx) / 2.0
    uf = np.zeros((3, fx * fy))
    uf[0] = A * np.sin(k * yf)
    fields = ((np.ones(Nc), u, None), (np.ones(fx * fy), uf, None))
    g0, g1, og, sim, _ = run_refined(case, 200, "f32", fields)
    _, uc = sim.moments(0)
    _, ufg = sim.moments(1)
    _, uco = og.coarse.moments()
    _, ufo = og.fine.moments()
    normal = og.crole == 0
    assert np.abs(uc.cpu().numpy()[0][normal] - uco[0][normal]).max() < 1e-6
    assert np.abs(ufg.cpu().numpy()[0] - ufo[0]).max() < 1e-6


def test_refined_layout_and_updates_per_step():
    case = dict(name="ref-set", q=9, shape=(32, 32, 1), lo=(8, 8, 0), hi=(20, 20, 0))
    sim = refined_sim(case, "f32")
    sim.init(level=0)
    sim.init(level=1)
    assert sim.levels == 2
    assert sim.updates_per_step == (32 * 32 - 11 * 11) + 2 * (25 * 25 - 4 * 24)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("noise", [True, False])
def test_refined_checkpoint_resume_bitwise(storage, noise):
    """Three levels with an inlet drawing noise (eager stepping) or without
    (graph replays of two coarse steps): 2n coarse steps equal n steps,
    checkpoint (time, populations of every level, interface records),
    restore into a fresh context initialised with other fields, n steps,
    bitwise on every level."""
    from tests.pair import multilevel_sim
    shape = (34, 26, 26)
    mask = W.jet_inlet_mask(*shape, D=6)
    case = dict(name="ml-ckpt", q=19, shape=shape, lo=(7, 6, 6), hi=(21, 19, 19),
                nest=[((6, 6, 6), (20, 20, 20))], tau=0.52, ma=0.2, seed=3,
                inlet_noise=0.02 if noise else 0.0, face_bc=(2, 2, 1, 1, 2, 2),
                sponge_width=(0, 8, 0, 0, 0, 4), chi_max=0.3, masks=[mask, None, None])
    n = 5
    sims = []
    for k in range(3):
        log("refined checkpoint storage=%s noise=%s sim %d" % (storage, noise, k))
        s = multilevel_sim(case, storage)
        for l in range(3):
            f = W.random_state(s.shape(l), seed=(40 if k < 2 else 90) + l, d=3, u_amp=0.03,
                               rho_amp=0.01, pi_amp=5e-4)
            s.init(*f, mask=case["masks"][l], level=l)
        sims.append(s)
    a, b, c = sims
    a.step(2 * n)
    b.step(n)
    ck = b.checkpoint()
    assert ck["time"] == n and len(ck["pops"]) == 3 and len(ck["interfaces"]) == 2
    c.restore(ck)
    assert c.time == n
    c.step(n)
    for l in range(3):
        np.testing.assert_array_equal(c.populations(l).cpu().numpy(),
                                      a.populations(l).cpu().numpy())
    assert c.time == a.time == 2 * n
    c.sync()


def test_interface_checkpoint_arguments():
    from paper_1710_02065_amd import lbm
    case = dict(name="ref-args", q=9, shape=(32, 32, 1), lo=(8, 8, 0), hi=(20, 20, 0))
    sim = refined_sim(case, "f32")
    sim.init(level=0)
    sim.init(level=1)
    nb = lbm.lbm_interface_bytes(sim.ctx, 0)
    assert nb == 2 * (13 + 2) * (13 + 2) * 10 * 4
    with pytest.raises(lbm.LbmError):
        lbm.lbm_interface_bytes(sim.ctx, 1)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_set_time(sim.ctx, -1)
    assert e.value.code == lbm.LBM_EINVAL


# ------------------------------------------------------------------------
# More than two levels: the coupling at every interface of a nested chain
# ------------------------------------------------------------------------
def run_multilevel(case, steps, storage="f64", seed=1):
    from tests.pair import multilevel_pair, multilevel_sim
    og = multilevel_pair(case)
    d = 2 if case["q"] == 9 else 3
    fields = [W.random_state(g.shape, seed=seed + l, d=d, u_amp=0.03, rho_amp=0.01,
                             pi_amp=5e-4) for l, g in enumerate(og.grids)]
    masks = case.get("masks") or [None] * len(og.grids)
    log("multilevel %s q=%d levels=%d shapes=%s storage=%s steps=%d"
        % (case.get("name"), case["q"], len(og.grids), [g.shape for g in og.grids], storage,
           steps))
    sim = multilevel_sim(case, storage)
    for l, f in enumerate(fields):
        sim.init(*f, mask=masks[l], level=l)
    sim.step(steps)
    pops = [sim.populations(l).cpu().numpy() for l in range(len(og.grids))]
    sim.sync()
    for l, f in enumerate(fields):
        og.init(l, *f)
    og.step(steps)
    return pops, og, sim


@pytest.mark.parametrize("q", [9, 19, 27])
def test_three_level_parity_f64(q):
    if q == 9:
        case = dict(name="ml2d", q=9, shape=(48, 40, 1), lo=(10, 8, 0), hi=(36, 30, 0),
                    nest=[((12, 10, 0), (34, 30, 0))], tau=0.57)
    else:
        case = dict(name="ml3d", q=q, shape=(24, 22, 20), lo=(5, 5, 5), hi=(17, 16, 15),
                    nest=[((6, 6, 6), (16, 15, 14))], tau=0.55)
    pops, og, sim = run_multilevel(case, 4)
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2  # COVERED nodes are never updated
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l
    assert sim.updates_per_step == sum(
        int(((og.crole[l] == 0) & (og.ring[l] == 0)).sum()) << l for l in range(3))


def test_four_level_2d_parity_f64():
    case = dict(name="ml4", q=9, shape=(40, 36, 1), lo=(8, 8, 0), hi=(30, 28, 0),
                nest=[((8, 8, 0), (36, 32, 0)), ((10, 10, 0), (46, 40, 0))], tau=0.6)
    pops, og, _ = run_multilevel(case, 3)
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l


FIVE_3D = dict(shape=(20, 20, 20), lo=(4, 4, 4), hi=(13, 13, 13),
               nest=[((4, 4, 4), (14, 14, 14)), ((4, 4, 4), (16, 16, 16)),
                     ((4, 4, 4), (20, 20, 20))])


@pytest.mark.parametrize("q", [19, 27])
def test_five_level_3d_parity_f64(q):
    """Level 0 and four nested boxes (the five levels of the jet setup of
    Sec. IV), every level against the oracle's multi-level driver."""
    case = dict(name="ml5-3d", q=q, tau=0.56, **FIVE_3D)
    pops, og, sim = run_multilevel(case, 2)
    assert len(og.grids) == 5
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l
    assert sim.updates_per_step == sum(
        int(((og.crole[l] == 0) & (og.ring[l] == 0)).sum()) << l for l in range(5))
    assert sim.time == 2


def test_five_level_2d_parity_f64():
    case = dict(name="ml5-2d", q=9, shape=(40, 36, 1), lo=(8, 8, 0), hi=(30, 28, 0),
                nest=[((8, 8, 0), (36, 32, 0)), ((10, 10, 0), (46, 40, 0)),
                      ((12, 12, 0), (60, 48, 0))], tau=0.58)
    pops, og, _ = run_multilevel(case, 3)
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l


def test_four_level_3d_parity_f64():
    case = dict(name="ml4-3d", q=19, shape=(22, 20, 20), lo=(5, 4, 4), hi=(16, 14, 15),
                nest=[((4, 4, 4), (17, 15, 17)), ((4, 5, 4), (22, 18, 22))], tau=0.6)
    pops, og, _ = run_multilevel(case, 3)
    assert len(og.grids) == 4
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l


def test_five_level_open_boundaries_parity_f64():
    """Five levels with an inlet disc drawing noise (counter blocks of five
    levels), an outflow layer and free-slip / outflow faces on level 0."""
    shape = (30, 22, 22)
    mask = W.jet_inlet_mask(*shape, D=6)
    box = ((4, 4, 4), (20, 18, 18))
    case = dict(name="ml5-open", q=19, shape=shape, lo=(5, 4, 4), hi=(20, 17, 17),
                nest=[box, box, box], tau=0.53, ma=0.2, seed=8, inlet_noise=0.02,
                face_bc=(2, 2, 1, 1, 2, 2), sponge_width=(0, 5, 0, 0, 0, 0), chi_max=0.3,
                masks=[mask, None, None, None, None])
    pops, og, _ = run_multilevel(case, 3)
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l


def test_three_level_open_boundaries_parity_f64():
    """Inlet disc with noise (counter blocks of three levels), sponge and
    free-slip/outflow faces on level 0, two nested boxes in the middle."""
    shape = (34, 26, 26)
    mask = W.jet_inlet_mask(*shape, D=6)
    case = dict(name="ml-open", q=19, shape=shape, lo=(7, 6, 6), hi=(21, 19, 19),
                nest=[((6, 6, 6), (20, 20, 20))], tau=0.52, ma=0.2, seed=3,
                inlet_noise=0.02, face_bc=(2, 2, 1, 1, 2, 2), sponge_width=(0, 8, 0, 0, 0, 4),
                chi_max=0.3, masks=[mask, None, None])
    pops, og, _ = run_multilevel(case, 5)
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l


def test_three_level_f32_tracks_oracle():
    """FP32 storage over three levels stays within the derived bound of the
    FP64 oracle (the two-level shear-wave argument, per level)."""
    case = dict(name="ml-f32", q=9, shape=(48, 40, 1), lo=(10, 8, 0), hi=(36, 30, 0),
                nest=[((12, 10, 0), (34, 30, 0))], tau=0.6)
    pops, og, sim = run_multilevel(case, 40, "f32")
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= 2e-6 * 40 ** 0.5, l


def test_refined_field_sponge_jet_reference_parity_f64():
    """Per-cell absorbing layers on a refined jet (Sec. IV: the outflow layer
    relaxes to the round-jet similarity field): on level 0 the face profile
    of the x+, y and z faces with the similarity velocity as reference, on
    level 1 a weak spherical layer; both against the oracle's per-cell
    layers on its multi-level driver, FP64 within 1e-12."""
    from paper_1710_02065_amd import layers, lbm
    shape = (34, 26, 26)
    mask = W.jet_inlet_mask(*shape, D=6)
    case = dict(name="ml-field-sponge", q=27, shape=shape, lo=(4, 7, 7), hi=(16, 18, 18),
                tau=0.53, ma=0.2, seed=5, inlet_noise=0.02, face_bc=(2, 2, 1, 1, 2, 2),
                masks=[mask, None])
    from tests.pair import multilevel_pair, multilevel_sim
    og = multilevel_pair(case)
    U = 0.2 / math.sqrt(3)
    # level 0: the face profile of the x+, y-, y+, z-, z+ faces (width 7)
    chi0 = layers.face_layer(shape, (0, 7, 7, 7, 7, 7), 0.25)
    rho0, u0 = layers.jet_reference(shape, 6.0, U, inlet=(0.0, None, None), core=2.0,
                                    rho_ref=1.002)
    fshape = og.grids[1].shape
    chi1 = layers.circular_layer(fshape, ((fshape[0] - 1) / 2, (fshape[1] - 1) / 2,
                                          (fshape[2] - 1) / 2), 6.0, 30.0, 0.1)
    N1 = int(np.prod(fshape))
    rho1 = np.full(N1, 0.999)
    u1 = np.zeros((3, N1))
    u1[0] = 0.5 * U
    fields = [W.random_state(g.shape, seed=21 + l, d=3, u_amp=0.03, rho_amp=0.01, pi_amp=5e-4)
              for l, g in enumerate(og.grids)]
    log("refined field sponge q=27 levels=2")
    sim = multilevel_sim(case, "f64", flags=lbm.LBM_SPONGE_FIELD)
    for l, f in enumerate(fields):
        sim.init(*f, mask=case["masks"][l], level=l)
    sim.set_sponge(chi0, rho0, u0, level=0)
    sim.set_sponge(chi1, rho1, u1, level=1)
    sim.step(5)
    pops = [sim.populations(l).cpu().numpy() for l in range(2)]
    sim.sync()
    og.grids[0].set_sponge(chi0, rho0, u0)
    og.grids[1].set_sponge(chi1, rho1, u1)
    for l, f in enumerate(fields):
        og.init(l, *f)
    og.step(5)
    for l, g in enumerate(og.grids):
        keep = og.crole[l] != 2
        assert normwise(pops[l][:, keep], g.f[:, keep]) <= F64_TOL, l
    # the layers acted: without them the run differs
    ref = multilevel_pair(case)
    for l, f in enumerate(fields):
        ref.init(l, *f)
    ref.step(5)
    assert normwise(ref.grids[0].f, og.grids[0].f) > 1e-6


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_refined_graph_replay_matches_eager(storage):
    """Refined contexts replay captured graphs of two coarse steps (both
    level-0 parities, open faces and a layer, three levels): every level
    bitwise equal to eager stepping after each call, including odd counts
    that leave a remainder and switch the parity between graphs."""
    from paper_1710_02065_amd import lbm
    from tests.pair import multilevel_pair, multilevel_sim
    case = dict(name="ml-graph", q=19, shape=(24, 22, 20), lo=(5, 5, 5), hi=(17, 16, 15),
                nest=[((6, 6, 6), (16, 15, 14))], tau=0.55, face_bc=(2, 2, 1, 1, 2, 2),
                sponge_width=(0, 4, 0, 0, 0, 0), chi_max=0.2)
    og = multilevel_pair(case)
    fields = [W.random_state(g.shape, seed=31 + l, d=3, u_amp=0.03, rho_amp=0.01, pi_amp=5e-4)
              for l, g in enumerate(og.grids)]
    log("refined graph replay storage=%s" % storage)
    a = multilevel_sim(case, storage)
    b = multilevel_sim(case, storage, flags=lbm.LBM_NO_GRAPH)
    for sim in (a, b):
        for l, f in enumerate(fields):
            sim.init(*f, level=l)
    for n in (3, 2, 5, 10, 1, 4):
        a.step(n)
        b.step(n)
        for l in range(len(og.grids)):
            np.testing.assert_array_equal(a.populations(l).cpu().numpy(),
                                          b.populations(l).cpu().numpy())
        assert a.time == b.time
    a.sync()
    b.sync()
