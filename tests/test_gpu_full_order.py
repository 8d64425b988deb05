"""Full recursive regularization (LBM_FULL_ORDER, Sec. II.A order n > 2) on
the GPU against the oracle's full-order grid, through the C ABI.  Bars as
in test_gpu_parity: FP64 within 1e-12 normwise; FP32 formats within 2e-6
and FP16-shifted within 2e-4 of one oracle step from the GPU's own stored
state; batched runs bitwise equal to solo runs."""
import math

import numpy as np
import pytest

from paper_1710_02065_amd import workloads as W
from tests.pair import gpu_sim, log, normwise, oracle_grid, run_both
from tests.test_gpu_parity import F64_TOL, RAGGED, TOL, channel_case, dim
from tests.test_gpu_refine import run_refined

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("q", [9, 27])
@pytest.mark.parametrize("steps", [0, 1, 7])
def test_full_periodic_parity_f64(q, steps):
    shape = RAGGED[q]
    rho, u, p = W.random_state(shape, seed=60 + q, d=dim(q), u_amp=0.08)
    case = dict(name="full-periodic", q=q, shape=shape, tau=0.53, full=True)
    gf, of, _, _ = run_both(case, steps, "f64", rho, u, p)
    assert normwise(gf, of) <= F64_TOL


@pytest.mark.parametrize("q", [9, 27])
def test_full_boundary_rules_parity_f64(q):
    case = dict(channel_case(q), full=True)
    U = case["ma"] / math.sqrt(3)
    rho, u = W.uniform_perturbed(case["shape"], U, (1, 0, 0), seed=3, rel_noise=1e-2, d=dim(q))
    gf, of, _, _ = run_both(case, 25, "f64", rho, u)
    assert normwise(gf, of) <= F64_TOL


def test_full_differs_from_third_order():
    """The switch reaches the kernels: one step of the two schemes from the
    same state differs by the fourth- to sixth-order terms."""
    case = dict(name="order-switch", q=27, shape=RAGGED[27], tau=0.53)
    rho, u, p = W.random_state(case["shape"], seed=5, d=3, u_amp=0.1)
    g3, _, _, _ = run_both(case, 1, "f64", rho, u, p)
    gf, _, _, _ = run_both(dict(case, full=True), 1, "f64", rho, u, p)
    assert normwise(gf, g3) > 1e-6


@pytest.mark.parametrize("q", [9, 27])
@pytest.mark.parametrize("storage", ["f32", "f32s", "f16s"])
def test_full_low_precision_single_step(q, storage):
    shape = RAGGED[q]
    rho, u, p = W.random_state(shape, seed=70 + q, d=dim(q))
    case = dict(name="full-lowprec", q=q, shape=shape, tau=0.52, full=True)
    log("full lowprec q=%d storage=%s" % (q, storage))
    sim = gpu_sim(case, storage)
    sim.init(rho, u, p)
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


@pytest.mark.parametrize("q", [9, 27])
def test_full_refined_parity_f64(q):
    if q == 9:
        case = dict(name="full-ref2d", q=9, shape=(48, 40, 1), lo=(12, 9, 0), hi=(30, 25, 0),
                    tau=0.57, full=True)
    else:
        case = dict(name="full-ref3d", q=27, shape=(22, 20, 18), lo=(6, 5, 5), hi=(14, 13, 12),
                    tau=0.55, full=True)
    g0, g1, og, _, _ = run_refined(case, 6)
    skip = og.crole == 2
    assert normwise(g0[:, ~skip], og.coarse.f[:, ~skip]) <= F64_TOL
    assert normwise(g1, og.fine.f) <= F64_TOL


def test_full_batch_equals_solo():
    """Full-order and third-order contexts batched together (two launch
    groups) match their solo runs bitwise."""
    from paper_1710_02065_amd import lbm
    cases = [dict(name="f0", q=9, shape=(64, 48, 1), tau=0.6, full=True),
             dict(name="t0", q=9, shape=(40, 52, 1), tau=0.6),
             dict(name="f1", q=9, shape=(37, 91, 1), tau=0.7, face_bc=(2, 2, 1, 1, 0, 0),
                  sponge_width=(0, 8, 0, 0, 0, 0), chi_max=0.2, full=True)]
    steps = [21, 34, 13]
    fields = [W.random_state(c["shape"], seed=80 + k, d=2) for k, c in enumerate(cases)]
    for storage in ("f32", "f16s"):
        log("full batch storage=%s" % storage)
        solo = [gpu_sim(c, storage).init(*f).step(n).populations().cpu().numpy()
                for c, f, n in zip(cases, fields, steps)]
        sims = [gpu_sim(c, storage).init(*f) for c, f in zip(cases, fields)]
        lbm.lbm_step_batch([s.ctx for s in sims], steps)
        for s, ref in zip(sims, solo):
            np.testing.assert_array_equal(s.populations().cpu().numpy(), ref)
