"""Batched stepping (lbm_step_batch) and served jobs against the FP64 oracle.

The batched launch advances many resident contexts at once: contexts are
grouped by lattice, storage, sweep path and workgroup size, each group walks
its (job, tile) list in a persistent kernel, and runs of 16 steps replay as
hipGraphs with the step index kept in device memory (a base that the graph
advances plus a per-launch offset).  These tests check each context of such
a batch element by element against oracle.Grid (the collision of Sec. II.A,
eq. optimizedLB, with the absorbing layer of Sec. II.C, eq. spongeLB):

* FP64 storage within 1e-12 normwise, over step counts above 16 that are not
  multiples of 16 (graph replays plus a tail of single launches), contexts
  already advanced before the batch (nonzero start time, which the inlet
  noise counter depends on), and a second batch call continuing the first;
* FP32 / FP32S / FP16S: one batched step from the GPU's own stored state
  within 2e-6 / 2e-6 / 2e-4 of one oracle step (the one-step bars of the
  solo sweep);
* served jobs (continuous batching through serve.Server): FP64 jobs within
  1e-12 of an oracle run of the whole job; FP32 and FP16S jobs within
  n * eps1 of it, n the job's steps and eps1 the one-step bar: each step
  adds at most eps1 of rounding, and on these stable runs the update does
  not amplify earlier differences (streaming permutes values; the
  collision keeps rho and j and scales the stress by 1 - 1/tau).
"""
import math

import numpy as np
import pytest

from paper_1710_02065_amd import workloads as W
import oracle as O
from tests.pair import gpu_sim, log, normwise, oracle_grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
TOL = {"f32": 2e-6, "f32s": 2e-6, "f16s": 2e-4}


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _walled_2d():
    nx, ny = 61, 29
    mask = W.cylinder_mask(nx, ny, 7, 20, 14)
    return dict(name="walled2d", q=9, shape=(nx, ny, 1), tau=0.57, ma=0.2,
                face_bc=(2, 2, 1, 1, 0, 0), sponge_width=(0, 12, 0, 0, 0, 0), chi_max=0.3,
                rho_ref=1.0, u_ref=(0.2 / math.sqrt(3), 0, 0), seed=21, inlet_noise=0.03,
                mask=mask)


def _jet_3d(q, full=False):
    shape = (19, 14, 13)
    mask = W.closed_box_mask(*shape)
    mask[W.jet_inlet_mask(*shape, D=5) == W.INLET] = W.INLET
    return dict(name="jet%d%s" % (q, "full" if full else ""), q=q, shape=shape, tau=0.53,
                ma=0.3, seed=17, inlet_noise=0.02, mask=mask, face_bc=(2, 2, 1, 1, 2, 2),
                sponge_width=(0, 5, 3, 3, 3, 3), chi_max=0.25, full=full)


def _channel_3d():
    nx, ny, nz = 23, 15, 11
    mask = np.tile(W.cylinder_mask(nx, ny, 4, 8, 7), nz)
    return dict(name="channel19", q=19, shape=(nx, ny, nz), tau=0.55, ma=0.15,
                face_bc=(2, 2, 1, 1, 2, 2), sponge_width=(0, 6, 0, 0, 3, 3), chi_max=0.3,
                rho_ref=1.0, u_ref=(0.15 / math.sqrt(3), 0, 0), seed=9, inlet_noise=0.05,
                mask=mask)


def batch_cases():
    """Mixed contexts: three lattices, periodic and general sweep paths,
    third and full order, masks, inlet noise, absorbing layers, ragged
    shapes (tails in every tile direction)."""
    return [
        dict(name="periodic2d", q=9, shape=(45, 37, 1), tau=0.53),
        _walled_2d(),
        dict(name="periodic2d-full", q=9, shape=(33, 70, 1), tau=0.58, full=True),
        dict(name="periodic19", q=19, shape=(17, 13, 11), tau=0.52),
        _channel_3d(),
        dict(name="periodic27", q=27, shape=(15, 12, 9), tau=0.6),
        _jet_3d(27, full=True),
        _jet_3d(27),
    ]


def _fields(case, seed):
    d = 2 if case["q"] == 9 else 3
    if case.get("mask") is not None:
        U = case.get("ma", 0.0) / math.sqrt(3)
        rho, u = W.uniform_perturbed(case["shape"], U, (1, 0, 0), seed=seed, rel_noise=2e-2, d=d)
        return rho, u, None
    return W.random_state(case["shape"], seed=seed, d=d)


def test_batch_f64_matches_oracle_with_graph_tail_and_offsets():
    from paper_1710_02065_amd import lbm
    cases = batch_cases()
    pre = [0, 3, 0, 5, 1, 0, 2, 7]          # solo steps before the batch
    first = [37, 21, 53, 16, 44, 5, 19, 0]  # graph replays + tails, one idle job
    second = [19, 40, 0, 33, 17, 2, 31, 23]  # the batch continues from there
    fields = [_fields(c, 70 + k) for k, c in enumerate(cases)]
    sims = []
    for c, f, n in zip(cases, fields, pre):
        log("batch f64 init %s" % c["name"])
        s = gpu_sim(c, "f64").init(*f, c.get("mask"))
        if n:
            s.step(n)
        sims.append(s)
    grids = [oracle_grid(c).init(*f) for c, f in zip(cases, fields)]
    for rnd, steps in enumerate((first, second)):
        log("batch f64 call %d steps=%s" % (rnd, steps))
        lbm.lbm_step_batch([s.ctx for s in sims], steps)
        for k, (c, s, g) in enumerate(zip(cases, sims, grids)):
            n = (pre[k] if rnd == 0 else 0) + steps[k]
            g.step(n)
            gf = s.populations().cpu().numpy()
            assert s.time == g.t, (c["name"], s.time, g.t)
            err = normwise(gf, g.f)
            assert err <= F64_TOL, (c["name"], rnd, err)
            if rnd == 1:
                r_g, u_g = s.moments()
                r_o, u_o = g.moments()
                assert normwise(r_g.cpu().numpy(), r_o) <= F64_TOL, c["name"]
                assert normwise(u_g.cpu().numpy(), u_o) <= F64_TOL, c["name"]


@pytest.mark.parametrize("storage", ["f32", "f32s", "f16s"])
def test_batch_narrow_single_step_matches_oracle(storage):
    """Contexts batched for n steps (graph replays and a tail), then one
    more batched step from the stored state, against one oracle step from
    that state (exactly converted)."""
    from paper_1710_02065_amd import lbm
    cases = batch_cases()
    steps = [37, 18, 21, 16, 40, 3, 17, 22]
    fields = [_fields(c, 90 + k) for k, c in enumerate(cases)]
    log("batch %s init" % storage)
    sims = [gpu_sim(c, storage).init(*f, c.get("mask")) for c, f in zip(cases, fields)]
    lbm.lbm_step_batch([s.ctx for s in sims], steps)
    f0 = [s.populations().cpu().numpy() for s in sims]
    log("batch %s one step" % storage)
    lbm.lbm_step_batch([s.ctx for s in sims], [1] * len(sims))
    for c, s, a, n in zip(cases, sims, f0, steps):
        f1 = s.populations().cpu().numpy()
        g = oracle_grid(c)
        g.set_populations(a)
        g.t = n
        g.step(1)
        err = normwise(f1, g.f)
        assert err <= TOL[storage], (c["name"], storage, err)


# ------------------------------------------------------------- serving --
def _oracle_for_job(be, job, mask):
    cfg = be.config(job)
    d = np.array(cfg.u_dir[:], dtype=float)
    U = cfg.ma / math.sqrt(3) * d / np.linalg.norm(d)
    U[2] = 0.0
    return O.Grid(9, cfg.nx, cfg.ny, 1, tau=cfg.tau, rho0=cfg.rho0, u_in=tuple(U),
                  face_bc=tuple(cfg.face_bc), sponge_width=tuple(cfg.sponge_width),
                  chi_max=cfg.chi_max, rho_ref=cfg.rho_ref, u_ref=tuple(cfg.u_ref),
                  seed=cfg.seed, inlet_noise=cfg.inlet_noise, mask=mask)


def test_served_jobs_match_oracle():
    """A Poisson stream of cylinder and pulse jobs in FP64, FP32 and FP16S
    storage served under a memory budget that forces queueing; every job's
    final populations and moments against an oracle run of that job."""
    from paper_1710_02065_amd import serve
    js = W.serving_jobs(12, 23, 1e6, side_range=(48, 144), step_range=(20, 90))
    kinds = ["cylinder", "pulse"]
    stores = ["f64", "f32", "f16s"]
    for k, j in enumerate(js):  # every (kind, storage) pair twice
        j["kind"] = kinds[k % 2]
        j["storage"] = stores[(k // 2) % 3]
    be = serve.GpuBackend(keep_populations=True)
    budget = sum(be.required_bytes(j) for j in js) // 3
    srv = serve.Server(be, budget, quantum=24)
    log("serving %d jobs, budget %d" % (len(js), budget))
    st = srv.run(js)
    assert st.summary()["jobs"] == len(js)
    assert any(r.admitted > r.job["arrival"] for r in srv.records)  # some queued
    seen = set()
    for r in srv.records:
        j = r.job
        rho0, u0, mask = r.result["init"]
        g = _oracle_for_job(be, j, mask).init(rho0, u0)
        g.step(j["steps"])
        gf = r.result["pops"].numpy()
        tol = F64_TOL if j["storage"] == "f64" else j["steps"] * TOL[j["storage"]]
        err = normwise(gf, g.f)
        assert err <= tol, (j["id"], j["kind"], j["storage"], j["steps"], err)
        r_o, _ = g.moments()
        err_r = normwise(r.result["rho"].numpy(), r_o)
        assert err_r <= tol, (j["id"], j["storage"], err_r)
        seen.add((j["kind"], j["storage"]))
    assert seen == {(k, s) for k in kinds for s in stores}
