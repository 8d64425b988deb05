"""lbm_step_batch_noalloc (job tables in a fixed device array, no
allocation) against lbm_step_batch through the C ABI: the two run the same
kernels, so every context's populations and time must agree bitwise, on
two calls in a row, the second with fewer and smaller contexts."""
import numpy as np
import pytest

from paper_1710_02065_amd import workloads as W
from tests.pair import gpu_sim, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cases():
    import math
    nx, ny = 61, 29
    mask = W.cylinder_mask(nx, ny, 7, 20, 14)
    walled = dict(name="walled2d", q=9, shape=(nx, ny, 1), tau=0.57, ma=0.2,
                  face_bc=(2, 2, 1, 1, 0, 0), sponge_width=(0, 12, 0, 0, 0, 0), chi_max=0.3,
                  u_ref=(0.2 / math.sqrt(3), 0, 0), seed=21, inlet_noise=0.03, mask=mask)
    shape = (19, 14, 13)
    jm = W.closed_box_mask(*shape)
    jm[W.jet_inlet_mask(*shape, D=5) == W.INLET] = W.INLET
    jet = dict(name="jet27", q=27, shape=shape, tau=0.53, ma=0.3, seed=17, inlet_noise=0.02,
               mask=jm, face_bc=(2, 2, 1, 1, 2, 2), sponge_width=(0, 5, 3, 3, 3, 3),
               chi_max=0.25)
    return [
        (dict(name="periodic2d", q=9, shape=(45, 37, 1), tau=0.53), "f64"),
        (walled, "f32"),
        (dict(name="periodic2d-full", q=9, shape=(33, 70, 1), tau=0.58, full=True), "f16s"),
        (dict(name="periodic19", q=19, shape=(17, 13, 11), tau=0.52), "f32"),
        (dict(name="periodic19b", q=19, shape=(30, 9, 5), tau=0.6), "f32"),
        (jet, "f64"),
        (dict(jet, name="jet27-f16s"), "f16s"),
        (dict(name="periodic27", q=27, shape=(15, 12, 9), tau=0.6), "f32s"),
    ]


def _make(cases, seed0):
    sims = []
    for k, (c, st) in enumerate(cases):
        d = 2 if c["q"] == 9 else 3
        if c.get("mask") is not None:
            rho, u = W.uniform_perturbed(c["shape"], 0.1, (1, 0, 0), seed=seed0 + k,
                                         rel_noise=2e-2, d=d)
            sims.append(gpu_sim(c, st).init(rho, u, None, c["mask"]))
        else:
            sims.append(gpu_sim(c, st).init(*W.random_state(c["shape"], seed=seed0 + k, d=d)))
    return sims


def _compare(a, b):
    for sa, sb in zip(a, b):
        assert sa.time == sb.time
        np.testing.assert_array_equal(sa.populations().cpu().numpy(),
                                      sb.populations().cpu().numpy())


def test_noalloc_batch_equals_batch_on_two_calls():
    from paper_1710_02065_amd import lbm
    cases = _cases()
    log("noalloc first call: %d contexts" % len(cases))
    a = _make(cases, 300)
    b = _make(cases, 300)
    steps = [37, 21, 53, 16, 5, 19, 0, 44]
    lbm.lbm_step_batch_noalloc([s.ctx for s in a], steps)
    lbm.lbm_step_batch([s.ctx for s in b], steps)
    _compare(a, b)
    log("noalloc second call: 3 smaller contexts")
    small = [(dict(c, name=c["name"] + "-small",
                   shape=tuple(max(1, v // 2) for v in c["shape"])), st)
             for c, st in cases if c.get("mask") is None][:3]
    a2 = _make(small, 400)
    b2 = _make(small, 400)
    steps2 = [7, 18, 3]
    lbm.lbm_step_batch_noalloc([s.ctx for s in a2], steps2)
    lbm.lbm_step_batch([s.ctx for s in b2], steps2)
    _compare(a2, b2)
    # the first contexts continue unchanged by the second call's tables
    lbm.lbm_step_batch_noalloc([s.ctx for s in a[:2]], [3, 1])
    lbm.lbm_step_batch([s.ctx for s in b[:2]], [3, 1])
    _compare(a, b)


def test_noalloc_batch_rejects_too_many_contexts():
    from paper_1710_02065_amd import lbm
    c = dict(name="one", q=9, shape=(8, 8, 1), tau=0.6)
    s = gpu_sim(c, "f32").init()
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_step_batch_noalloc([s.ctx] * (lbm.LBM_NOALLOC_MAX_JOBS + 1),
                                   [1] * (lbm.LBM_NOALLOC_MAX_JOBS + 1))
    assert e.value.code == lbm.LBM_EINVAL
    assert "at most %d" % lbm.LBM_NOALLOC_MAX_JOBS in lbm.lbm_last_error()
    assert s.time == 0
