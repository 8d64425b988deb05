"""The comparator collisions (LBM_BGK on every lattice, LBM_MRT on D2Q9;
Sec. II.A) on the GPU against the oracle's comparator grids, through the
C ABI: FP64 within 1e-12 normwise, narrow formats to the bars of
test_gpu_parity for one step from the GPU's own state."""
import math

import numpy as np
import pytest

from paper_1710_02065_amd import workloads as W
from tests.pair import gpu_sim, log, normwise, oracle_grid
from tests.test_gpu_parity import F64_TOL, RAGGED, TOL, channel_case, dim

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FLAG = {"bgk": 0x10, "mrt": 0x20}


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_pair(case, collision, steps, storage="f64", rho=None, u=None, p=None):
    log("%s %s q=%d storage=%s steps=%d" % (collision, case["name"], case["q"], storage, steps))
    sim = gpu_sim(case, storage, flags=FLAG[collision])
    sim.init(rho, u, p, case.get("mask"))
    sim.step(steps)
    gf = sim.populations().cpu().numpy()
    sim.sync()
    g = oracle_grid(case)
    g = type(g)(case["q"], *case["shape"], tau=g.g.tau, rho0=g.g.rho0,
                u_in=tuple(g.g.u_in), face_bc=tuple(g.g.face_bc),
                sponge_width=tuple(g.g.sponge_width), chi_max=g.g.chi_max,
                rho_ref=g.g.rho_ref, u_ref=tuple(g.g.u_ref), seed=g.g.seed,
                inlet_noise=g.g.inlet_noise, mask=case.get("mask"), collision=collision)
    g.init(rho, u, p).step(steps)
    return gf, g.f


@pytest.mark.parametrize("q", [9, 19, 27])
def test_bgk_periodic_parity_f64(q):
    rho, u, p = W.random_state(RAGGED[q], seed=110 + q, d=dim(q), u_amp=0.05)
    case = dict(name="bgk-periodic", q=q, shape=RAGGED[q], tau=0.53)
    gf, of = run_pair(case, "bgk", 7, "f64", rho, u, p)
    assert normwise(gf, of) <= F64_TOL


@pytest.mark.parametrize("q", [9, 19])
def test_bgk_channel_parity_f64(q):
    """Inlet with noise, free-slip, outflow, sponge and a body under BGK."""
    case = channel_case(q)
    U = case["ma"] / math.sqrt(3)
    rho, u = W.uniform_perturbed(case["shape"], U, (1, 0, 0), seed=6, rel_noise=1e-2, d=dim(q))
    gf, of = run_pair(case, "bgk", 20, "f64", rho, u)
    assert normwise(gf, of) <= F64_TOL


def test_mrt_parity_f64():
    rho, u, p = W.random_state(RAGGED[9], seed=120, d=2, u_amp=0.05)
    case = dict(name="mrt-periodic", q=9, shape=RAGGED[9], tau=0.52)
    gf, of = run_pair(case, "mrt", 7, "f64", rho, u, p)
    assert normwise(gf, of) <= F64_TOL
    # walls and a body (no sponge: the MRT comparator has none)
    shape = (64, 40, 1)
    mask = W.cylinder_mask(64, 40, 10, 20, 20)
    case = dict(name="mrt-channel", q=9, shape=shape, tau=0.55, ma=0.15, face_bc=(2, 2, 1, 1, 0, 0),
                mask=mask)
    rho, u = W.uniform_perturbed(shape, 0.08, (1, 0, 0), seed=8, rel_noise=1e-2, d=2)
    gf, of = run_pair(case, "mrt", 15, "f64", rho, u)
    assert normwise(gf, of) <= F64_TOL


@pytest.mark.parametrize("collision,q", [("bgk", 19), ("bgk", 27), ("mrt", 9)])
@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_comparator_low_precision_single_step(collision, q, storage):
    shape = RAGGED[q]
    rho, u, p = W.random_state(shape, seed=130 + q, d=dim(q))
    case = dict(name="cmp-lowprec", q=q, shape=shape, tau=0.52)
    log("%s lowprec q=%d storage=%s" % (collision, q, storage))
    sim = gpu_sim(case, storage, flags=FLAG[collision])
    sim.init(rho, u, p)
    sim.step(2)
    f0 = sim.populations().cpu().numpy()
    sim.step(1)
    f1 = sim.populations().cpu().numpy()
    sim.sync()
    from oracle import Grid
    g = Grid(q, *shape, tau=0.52, collision=collision)
    g.set_populations(f0)
    g.t = 2
    g.step(1)
    assert normwise(f1, g.f) <= TOL[storage]
