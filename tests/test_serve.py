"""Serving scheduler on the CPU with a simulated clock (FakeBackend), and
on the GPU: each job's result is bitwise the same alone and in the mix."""
import numpy as np
import pytest

from paper_1710_02065_amd import serve
from paper_1710_02065_amd import workloads as W


def jobs(n=40, seed=5, rate=50.0, scale=0.02):
    return W.serving_jobs(n, seed, rate, step_scale=scale)


def test_budget_never_exceeded_and_all_jobs_finish():
    js = jobs()
    be = serve.FakeBackend(mlups=2000.0)
    budget = 3 * max(be.required_bytes(j) for j in js)
    st = serve.Server(be, budget, quantum=64).run(js)
    assert len(st.latencies) == len(js)
    assert be.max_live_bytes <= budget
    assert st.peak_bytes <= budget
    assert not be.live
    # every job received exactly its step count
    total = {}
    for call in be.calls:
        for jid, n in call:
            total[jid] = total.get(jid, 0) + n
    assert total == {j["id"]: j["steps"] for j in js}


@pytest.mark.parametrize("lookahead", [0, 1, 2])
def test_lookahead_keeps_budget_and_steps(lookahead):
    """With quanta queued ahead of the one the host waits for, a job's memory
    returns to the budget only once its last quantum has completed, every
    job still receives exactly its steps, and the budget holds."""
    js = jobs(n=30, rate=200.0)
    be = serve.FakeBackend(mlups=2000.0)
    budget = 3 * max(be.required_bytes(j) for j in js)
    st = serve.Server(be, budget, quantum=64, lookahead=lookahead).run(js)
    assert len(st.latencies) == len(js)
    assert be.max_live_bytes <= budget and st.peak_bytes <= budget
    total = {}
    for call in be.calls:
        for jid, n in call:
            total[jid] = total.get(jid, 0) + n
    assert total == {j["id"]: j["steps"] for j in js}
    assert not be.live


def test_queueing_grows_with_load():
    out = []
    for rate in (5.0, 500.0):
        js = jobs(rate=rate)
        be = serve.FakeBackend(mlups=2000.0)
        budget = 4 * max(be.required_bytes(j) for j in js)
        out.append(serve.Server(be, budget, quantum=64).run(js).summary())
    assert out[1]["p50_queue_s"] >= out[0]["p50_queue_s"]
    assert out[1]["p99_latency_s"] >= out[0]["p50_latency_s"]


def test_admission_in_arrival_order_when_everything_fits():
    js = jobs(n=12, rate=1000.0)
    be = serve.FakeBackend()
    srv = serve.Server(be, 10 ** 15, quantum=32)
    srv.run(js)
    recs = srv.records
    for a in recs:
        for b in recs:
            if a.job["arrival"] < b.job["arrival"]:
                assert a.admitted <= b.admitted
    # a job cannot finish faster than its own work at the full throughput
    for r in recs:
        assert r.finished - r.job["arrival"] >= be.cells(r.job) * r.job["steps"] / 1e9 - 1e-12


def _stream_with_big_job(n_small, big_at=5):
    """Short 64x64 jobs arriving faster than they finish, and one 256x256
    job (the whole budget) arriving as the sixth."""
    js = []
    t = 0.0
    for k in range(n_small + 1):
        big = k == big_at
        js.append(dict(id=k, kind="pulse", nx=256 if big else 64, ny=256 if big else 64,
                       ma=0.1, steps=300 if big else 200, storage="f32", seed=k, arrival=t))
        t += 2e-4
    return js


@pytest.mark.parametrize("n_small", [40, 400])
def test_reserved_head_job_is_not_starved(n_small):
    """Tight budget: the large job needs all of it.  Later small jobs are
    admitted past it only if they end before it can start, so its queueing
    delay is bounded by the work resident when it reached the head of the
    queue (at most one small job's steps), independent of how long the
    stream of small jobs lasts."""
    js = _stream_with_big_job(n_small)
    be = serve.FakeBackend(mlups=2000.0, launch_overhead=1e-4)
    big = max(js, key=lambda j: j["nx"] * j["ny"])
    budget = be.required_bytes(big)
    srv = serve.Server(be, budget, quantum=50)
    st = srv.run(js)
    assert len(st.latencies) == len(js)
    assert be.max_live_bytes <= budget
    rec = {r.job["id"]: r for r in srv.records}[big["id"]]
    small_steps = max(j["steps"] for j in js if j is not big)
    calls = -(-small_steps // 50)  # batched calls until the resident jobs end
    per_call = 1e-4 + (budget / be.bpc) * 50 / (be.mlups * 1e6)  # a full budget's quantum
    assert rec.admitted - big["arrival"] <= calls * per_call + 1e-12


def test_job_larger_than_budget_is_rejected():
    js = jobs(n=3)
    be = serve.FakeBackend()
    with pytest.raises(ValueError):
        serve.Server(be, 10, quantum=16).run(js)


def test_percentiles():
    v = list(range(1, 101))
    assert serve.Stats.pct(v, 50) == pytest.approx(50.5)
    assert serve.Stats.pct(v, 99) == pytest.approx(99.01)


@pytest.mark.gpu
def test_gpu_results_same_alone_and_in_mix():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    js = W.serving_jobs(6, 11, 1e6, side_range=(96, 320), step_range=(40, 200))
    be = serve.GpuBackend(keep_populations=True)
    budget = sum(be.required_bytes(j) for j in js) // 2  # forces queueing
    srv = serve.Server(be, budget, quantum=48)
    st = srv.run(js)
    assert st.summary()["jobs"] == len(js)
    mixed = {r.job["id"]: r.result["pops"].numpy() for r in srv.records}
    for j in js:
        h = be.start(j)
        be.lbm.lbm_step(h["ctx"], j["steps"])
        alone = be.finish(h)["pops"].numpy()
        np.testing.assert_array_equal(alone, mixed[j["id"]])
