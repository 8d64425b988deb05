"""Slab decomposition through the C ABI (face rule LBM_HALO, halo buffers
and exchange): one grid split along its last axis into subdomains that
exchange the populations crossing each cut after every step.

Bars: bitwise equality of every population with the undivided grid stepped
on the same sweep path, for every storage format (slabs of a grid whose other
faces are periodic and that has no mask stay on the periodic path; a mask,
even all FLUID, or another face rule selects the general path for both); the
FP64 split run within 1e-12 of the oracle; the documented send-buffer
layout exactly.
"""
import numpy as np
import pytest

from paper_1710_02065_amd import lbm
from paper_1710_02065_amd import workloads as W
from paper_1710_02065_amd.slabs import Slabs
from tests.pair import gpu_sim, log, normwise, oracle_grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def undivided(case, storage, mask=None, fields=(None, None, None), steps=0):
    sim = gpu_sim(case, storage)
    sim.init(*fields, mask)
    sim.step(steps)
    return sim


def split_run(case, k, storage, mask=None, fields=(None, None, None), steps=0):
    kw = dict(lattice=case["q"], tau=case.get("tau", 0.6), storage=storage,
              rho0=case.get("rho0", 1.0), ma=case.get("ma", 0.0),
              u_dir=case.get("u_dir", (1.0, 0.0, 0.0)), face_bc=case.get("face_bc", (0,) * 6),
              sponge_width=case.get("sponge_width", (0,) * 6), chi_max=case.get("chi_max", 0.0),
              rho_ref=case.get("rho_ref", 1.0), u_ref=case.get("u_ref", (0.0, 0.0, 0.0)),
              flags=lbm.LBM_FULL_ORDER if case.get("full") else 0)
    sl = Slabs(k, case["shape"], **kw)
    sl.init(*fields, mask)
    sl.step(steps)
    return sl


def same(a, b):
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("storage", ["f64", "f32", "f32s", "f16s"])
@pytest.mark.parametrize("k", [1, 2, 4])
@pytest.mark.parametrize("general", [False, True])
def test_periodic_ring_matches_undivided_bitwise(storage, k, general):
    """D3Q19 periodic grid as a ring of k slabs (k = 1: a context that is
    its own neighbour through both cuts), on the periodic path and, with an
    all-FLUID mask, on the general path."""
    case = dict(name="ring", q=19, shape=(40, 24, 12), tau=0.53)
    fields = W.random_state(case["shape"], seed=70 + k, d=3)
    mask = np.zeros(40 * 24 * 12, np.uint8) if general else None
    log("slab ring %s k=%d storage=%s general=%s" % (case["shape"], k, storage, general))
    ref = undivided(case, storage, mask=mask, fields=fields, steps=9)
    sl = split_run(case, k, storage, mask=mask, fields=fields, steps=9)
    assert same(sl.populations(), ref.populations())
    r1, u1 = sl.moments()
    r2, u2 = ref.moments()
    assert same(r1, r2) and same(u1, u2)
    sl.sync()
    ref.sync()
    sl.close()


@pytest.mark.parametrize("q,shape,k", [(9, (70, 45, 1), 3), (9, (33, 2, 1), 2),
                                       (27, (22, 14, 15), 3), (27, (9, 5, 2), 2)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_periodic_path_rings_d2q9_d3q27_bitwise(q, shape, k, storage):
    """Rings on the periodic path for D2Q9 (cut along y, three crossing
    directions) and D3Q27 (nine), including one-plane slabs, against the
    undivided periodic grid."""
    case = dict(name="ring%d" % q, q=q, shape=shape, tau=0.56)
    fields = W.random_state(shape, seed=94 + q + k, d=2 if q == 9 else 3)
    log("slab ring q=%d %s k=%d storage=%s" % (q, shape, k, storage))
    ref = undivided(case, storage, fields=fields, steps=7)
    sl = split_run(case, k, storage, fields=fields, steps=7)
    assert not sl.general
    assert same(sl.populations(), ref.populations())
    sl.sync()
    sl.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_channel_split_across_walls_bitwise(storage):
    """D2Q9 cylinder channel cut along y into three slabs: free-slip walls
    at the outer y faces (corner links across a cut and a wall), inlet
    column, outflow face with an absorbing layer, SOLID disc inside the
    middle slab."""
    nx, ny = 96, 64
    mask = W.cylinder_mask(nx, ny, 6, 30, 32)
    mask[::nx] = lbm.LBM_INLET
    case = dict(name="channel", q=9, shape=(nx, ny, 1), tau=0.56, ma=0.2,
                face_bc=(2, 2, 1, 1, 0, 0), sponge_width=(0, 16, 0, 0, 0, 0), chi_max=0.2,
                u_ref=(0.2 * 3 ** -0.5, 0.0, 0.0))
    log("slab channel storage=%s" % storage)
    ref = undivided(case, storage, mask=mask, steps=60)
    sl = split_run(case, 3, storage, mask=mask, steps=60)
    assert sl.sizes == [22, 21, 21]
    assert same(sl.populations(), ref.populations())
    sl.sync()
    sl.close()


@pytest.mark.parametrize("full", [False, True])
def test_d3q27_open_chain_bitwise(full):
    """D3Q27 chain of three slabs with outflow / free-slip ends along z,
    outflow x faces with an absorbing layer, periodic y."""
    case = dict(name="chain27", q=27, shape=(28, 10, 21), tau=0.55, ma=0.1,
                face_bc=(2, 2, 0, 0, 2, 1), sponge_width=(0, 8, 0, 0, 0, 0), chi_max=0.3,
                full=full)
    fields = W.random_state(case["shape"], seed=81, d=3)
    log("slab chain D3Q27 full=%s" % full)
    ref = undivided(case, "f32", mask=np.zeros(28 * 10 * 21, np.uint8), fields=fields, steps=7)
    sl = split_run(case, 3, "f32", mask=np.zeros(28 * 10 * 21, np.uint8), fields=fields,
                   steps=7)
    assert same(sl.populations(), ref.populations())
    sl.sync()
    sl.close()


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_open_ends_split_bitwise(storage):
    """Periodic x and y, outflow z ends, no mask: the undivided grid runs the
    general path, and so does every slab (the middle one included, whose
    faces are all periodic or cuts), so the split run stays bitwise equal."""
    case = dict(name="open-ends", q=19, shape=(32, 20, 18), tau=0.55, ma=0.05,
                face_bc=(0, 0, 0, 0, 2, 2))
    fields = W.random_state(case["shape"], seed=93, d=3)
    log("slab open ends storage=%s" % storage)
    ref = undivided(case, storage, fields=fields, steps=8)
    sl = split_run(case, 3, storage, fields=fields, steps=8)
    assert sl.general
    assert same(sl.populations(), ref.populations())
    sl.sync()
    sl.close()


@pytest.mark.parametrize("q,flags,faces,shape", [
    (9, lbm.LBM_MRT, (0, 0, 0, 0, 0, 0), (48, 30, 1)),
    (9, lbm.LBM_BGK, (2, 2, 1, 1, 0, 0), (48, 30, 1)),
    (19, lbm.LBM_BGK, (0, 0, 0, 0, 2, 1), (20, 12, 15)),
    (27, lbm.LBM_BGK, (1, 1, 0, 0, 0, 0), (14, 10, 12))])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_comparator_collisions_split_bitwise(q, flags, faces, shape, storage):
    """The comparator collisions (LBM-BGK, D2Q9 LBM-MRT) across cuts: the
    halo pull is shared, so split runs stay bitwise the undivided ones."""
    case = dict(name="comparator", q=q, shape=shape, tau=0.6, face_bc=faces)
    fields = W.random_state(shape, seed=95 + q, d=2 if q == 9 else 3)
    n = int(np.prod(shape))
    mask = np.zeros(n, np.uint8)
    log("slab comparator q=%d flags=%d storage=%s" % (q, flags, storage))
    ref = gpu_sim(case, storage, flags=flags)
    ref.init(*fields, mask)
    ref.step(6)
    sl = Slabs(3, shape, lattice=q, tau=0.6, storage=storage, face_bc=faces, flags=flags)
    sl.init(*fields, mask)
    sl.step(6)
    assert same(sl.populations(), ref.populations())
    sl.sync()
    sl.close()


def test_split_run_matches_oracle_f64():
    """The split FP64 run against the undivided oracle grid."""
    case = dict(name="oracle", q=19, shape=(18, 11, 14), tau=0.57, face_bc=(1, 1, 0, 0, 2, 2),
                ma=0.05)
    fields = W.random_state(case["shape"], seed=90, d=3)
    log("slab oracle parity")
    sl = split_run(case, 3, "f64", fields=fields, steps=6)
    gf = sl.populations().cpu().numpy()
    sl.sync()
    sl.close()
    g = oracle_grid(case).init(*fields).step(6)
    assert normwise(gf, g.f) <= 1e-12


def test_send_buffer_layout():
    """Send buffers hold the face plane's leaving populations, row k = rank
    of the direction among those with the same last-axis component (read
    back through a caller-owned buffer bound as the context memory)."""
    case = dict(name="layout", q=19, shape=(16, 9, 6), tau=0.6)
    fields = W.random_state(case["shape"], seed=91, d=3)
    sim = gpu_sim(case, "f64", face_bc=(0, 0, 0, 0, 3, 3))
    nbytes = lbm.lbm_required_bytes(sim.cfg)
    mem = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    lbm.lbm_bind_memory(sim.ctx, mem, nbytes)
    sim.init(*fields)
    f = sim.populations().cpu().numpy().reshape(19, 6, 9, 16)
    xi, _ = lbm.lbm_lattice_table(19)
    plane = 16 * 9
    for side, zl, sign in [(0, 0, -1), (1, 5, 1)]:
        send, recv, nb = lbm.lbm_halo_buffers(sim.ctx, side)
        dirs = [i for i in range(19) if xi[i, 2] == sign]
        assert nb == len(dirs) * plane * 8 == 5 * plane * 8
        off = send - mem.data_ptr()
        assert 0 <= off and off + nb <= nbytes
        got = mem[off:off + nb].view(torch.float64).cpu().numpy().reshape(len(dirs), 9, 16)
        for k, i in enumerate(dirs):
            assert np.array_equal(got[k], f[i, zl]), (side, i)
        # before any exchange the receive buffer holds the own face plane's
        # entering populations (a zero-gradient face)
        offr = recv - mem.data_ptr()
        gotr = mem[offr:offr + nb].view(torch.float64).cpu().numpy().reshape(len(dirs), 9, 16)
        back = [i for i in range(19) if xi[i, 2] == -sign]
        for k, i in enumerate(back):
            assert np.array_equal(gotr[k], f[i, zl]), (side, i)
    sim.sync()
    sim.close()


def test_halo_contexts_step_once_per_call_and_refuse_batching():
    sim = gpu_sim(dict(q=19, shape=(8, 8, 4), tau=0.6), "f32", face_bc=(0, 0, 0, 0, 3, 3))
    sim.init()
    with pytest.raises(lbm.LbmError) as e:
        sim.step(2)
    assert "one step per call" in str(e.value)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_step_batch([sim.ctx], [1])
    assert e.value.code == lbm.LBM_EUNSUPPORTED
    other = gpu_sim(dict(q=19, shape=(8, 8, 4), tau=0.6), "f32")
    other.init()
    with pytest.raises(lbm.LbmError):
        lbm.lbm_halo_buffers(other.ctx, 0)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_halo_exchange([sim.ctx, other.ctx], False)
    sim.sync()


def test_solid_cell_on_cut_plane_rejected():
    sim = gpu_sim(dict(q=9, shape=(16, 12, 1), tau=0.6), "f32", face_bc=(0, 0, 3, 3, 0, 0))
    mask = np.zeros(16 * 12, np.uint8)
    mask[16 * 11 + 5] = lbm.LBM_SOLID
    with pytest.raises(lbm.LbmError) as e:
        sim.init(mask=mask)
    assert "halo face" in str(e.value)


def test_checkpoint_resume_across_cuts():
    """Populations taken from the split run and set into a new split run
    continue bitwise like the original."""
    case = dict(name="resume", q=19, shape=(24, 16, 20), tau=0.52, ma=0.1)
    fields = W.random_state(case["shape"], seed=92, d=3)
    log("slab checkpoint")
    a = split_run(case, 4, "f32", fields=fields, steps=5)
    f = a.populations()
    a.step(6)
    b = split_run(case, 4, "f32", fields=fields, steps=0)
    b.set_populations(f)
    b.step(6)
    assert same(a.populations(), b.populations())
    a.sync()
    b.sync()


def test_full_size_channel_in_three_slabs_bitwise():
    """The 2048 x 1024 cylinder channel (D = 100 at (400, 512), Ma 0.2, Re
    150, inlet column, outflow with a 128-column layer, free-slip walls) cut
    along y into three slabs whose cuts miss the disc, FP32, without inlet
    noise: equal to the undivided channel after 50 steps."""
    nx, ny, D = 2048, 1024, 100
    U = 0.2 * 3 ** -0.5
    case = dict(name="channel-full", q=9, shape=(nx, ny, 1), tau=0.5 + 3 * U * D / 150, ma=0.2,
                face_bc=(2, 2, 1, 1, 0, 0), sponge_width=(0, 128, 0, 0, 0, 0), chi_max=0.2,
                u_ref=(U, 0.0, 0.0))
    mask = W.cylinder_mask(nx, ny, D, 400, 512)
    rho, u = W.uniform_perturbed((nx, ny, 1), U, (1, 0, 0), seed=2, rel_noise=1e-4, d=2)
    log("slab full-size channel")
    sl = split_run(case, 3, "f32", mask=mask, fields=(rho, u, None), steps=50)
    assert sl.sizes == [342, 341, 341]
    got = sl.populations()
    sl.sync()
    sl.close()
    ref = undivided(case, "f32", mask=mask, fields=(rho, u, None), steps=50)
    assert same(got, ref.populations())
    ref.sync()


def test_headline_grid_in_eight_slabs_bitwise():
    """D3Q19 256^3 Taylor-Green + pulse (FP32) as eight 256x256x32 slabs,
    one GPU's share each when the grid is spread over eight GPUs: equal to
    the undivided grid (both on the periodic path) after 20 steps."""
    n = 256
    rho, u = W.taylor_green_3d(n, 0.0577, pulse_amp=1e-3)
    case = dict(name="headline", q=19, shape=(n, n, n), tau=0.52)
    log("slab headline 256^3 k=8")
    sl = split_run(case, 8, "f32", fields=(rho, u, None), steps=20)
    assert sl.sizes == [32] * 8
    got = sl.populations()
    sl.sync()
    sl.close()
    del sl
    ref = undivided(case, "f32", fields=(rho, u, None), steps=20)
    assert same(got, ref.populations())
    ref.sync()
