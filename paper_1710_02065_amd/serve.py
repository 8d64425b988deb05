"""Continuous-batching serving of many small lattices on one GPU.

Jobs (2D D2Q9 cylinder-in-channel or acoustic-pulse lattices of uneven
sizes) arrive over time.  The server keeps every admitted job's populations
resident in HBM, admits queued jobs in arrival order whenever their device
footprint (lbm_required_bytes) fits the remaining budget (a job that does
not fit is not overtaken by later jobs that would delay it), and advances all
resident jobs together: each quantum is one lbm_step_batch call, i.e. one
persistent batched launch sequence (replayed as hipGraphs) over the (job,
tile) work list of every resident lattice.  Jobs that arrive while others
run join at the next quantum; finished jobs release their memory at once.

Backends: `GpuBackend` drives the HIP library; `FakeBackend` is a
cost-model stand-in with a simulated clock for testing the scheduler on a
machine without a GPU.
"""
import math
import time
from dataclasses import dataclass, field

CS = math.sqrt(1.0 / 3.0)


@dataclass
class JobRecord:
    job: dict
    need: int = 0
    admitted: float = -1.0
    finished: float = -1.0
    done_steps: int = 0
    handle: object = None
    result: object = None

    @property
    def remaining(self):
        return self.job["steps"] - self.done_steps


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    queue_delays: list = field(default_factory=list)
    cell_updates: int = 0
    makespan: float = 0.0
    peak_bytes: int = 0
    quanta: int = 0

    @staticmethod
    def pct(values, p):
        if not values:
            return float("nan")
        v = sorted(values)
        k = (len(v) - 1) * p / 100.0
        f = math.floor(k)
        c = min(f + 1, len(v) - 1)
        return v[f] + (v[c] - v[f]) * (k - f)

    def summary(self):
        return dict(jobs=len(self.latencies),
                    p50_latency_s=self.pct(self.latencies, 50),
                    p99_latency_s=self.pct(self.latencies, 99),
                    p50_queue_s=self.pct(self.queue_delays, 50),
                    p99_queue_s=self.pct(self.queue_delays, 99),
                    mlups=self.cell_updates / self.makespan / 1e6 if self.makespan > 0 else 0.0,
                    makespan_s=self.makespan, peak_bytes=self.peak_bytes, quanta=self.quanta)


class Server:
    """Admission + continuous batching loop.

    budget_bytes: HBM budget for resident jobs; quantum: steps per batched
    call (a job near its end takes only its remaining steps); lookahead:
    batched calls enqueued beyond the one the host waits for.  With
    lookahead 1 the next quantum is on the device while the host retires
    the jobs of the previous one and admits new ones, so the device does
    not idle between quanta; a job's memory returns to the budget once its
    last quantum has completed."""

    def __init__(self, backend, budget_bytes, quantum=256, lookahead=1):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.quantum = int(quantum)
        self.lookahead = int(lookahead)

    def run(self, jobs):
        be = self.backend
        pending = sorted((JobRecord(j) for j in jobs), key=lambda r: r.job["arrival"])
        for r in pending:
            r.need = be.required_bytes(r.job)
            if r.need > self.budget:
                raise ValueError("job %s needs %d bytes, more than the budget %d"
                                 % (r.job["id"], r.need, self.budget))
        queue, active, done = [], [], []
        inflight = []  # (completion mark, jobs whose last quantum it closes)
        used = 0
        st = Stats()
        t0 = be.now()
        while pending or queue or active or inflight:
            now = be.now() - t0
            while pending and pending[0].job["arrival"] <= now:
                queue.append(pending.pop(0))
            # Admit in arrival order.  The first queued job that does not fit
            # holds a reservation: a later job is admitted past it only if it
            # fits now and ends no later than the reserved job could start,
            # so the reserved job's wait is bounded by the work resident when
            # it reached the head of the queue, whatever arrives after it.
            wait = None  # steps until the reserved job fits
            for r in list(queue):
                if used + r.need > self.budget:
                    if wait is None:
                        retiring = [x for _, fin in inflight for x in fin]
                        wait = self._steps_until_fits(active + retiring, used, r.need)
                    continue
                if wait is not None and r.job["steps"] > wait:
                    continue
                r.handle = be.start(r.job)
                r.admitted = be.now() - t0
                used += r.need
                queue.remove(r)
                active.append(r)
            st.peak_bytes = max(st.peak_bytes, used)
            if active:
                steps = [min(self.quantum, r.remaining) for r in active]
                be.step([r.handle for r in active], steps)
                st.quanta += 1
                for r, n in zip(active, steps):
                    r.done_steps += n
                fin = [r for r in active if r.remaining == 0]
                for r in fin:
                    # results read out behind this quantum, collected later
                    r.result = be.retire(r.handle)
                    active.remove(r)
                inflight.append((be.mark(), fin))
            # wait for the oldest quantum once `lookahead` more are queued
            # behind it (or nothing more can be queued)
            while inflight and (len(inflight) > self.lookahead or not active):
                mark, fin = inflight.pop(0)
                be.wait(mark)
                for r in fin:
                    r.result = be.collect(r.handle, r.result)
                    r.finished = be.now() - t0
                    used -= r.need
                    done.append(r)
                    st.latencies.append(r.finished - r.job["arrival"])
                    st.queue_delays.append(r.admitted - r.job["arrival"])
                    st.cell_updates += be.cells(r.job) * r.job["steps"]
                if active:
                    break
            if not active and not inflight:
                be.idle()
                if pending and not queue:
                    be.wait_until(t0 + pending[0].job["arrival"])
        be.idle()
        if done:
            st.makespan = max(r.finished for r in done) - min(r.job["arrival"] for r in done)
        self.records = done
        return st


    def _steps_until_fits(self, active, used, need):
        """Steps after which a job of `need` bytes fits: every resident job
        advances by the same steps per batched call (up to its remaining
        steps), so they finish in the order of their remaining steps."""
        free = self.budget - used
        for r in sorted(active, key=lambda r: r.remaining):
            free += r.need
            if free >= need:
                return r.remaining
        return 0


class FakeBackend:
    """Scheduler test double: fixed throughput, simulated clock, no GPU."""

    def __init__(self, mlups=1000.0, bytes_per_cell=72, launch_overhead=1e-4):
        self.mlups = mlups
        self.bpc = bytes_per_cell
        self.overhead = launch_overhead
        self.clock = 0.0
        self.live = {}
        self.max_live_bytes = 0
        self.calls = []

    def now(self):
        return self.clock

    def wait_until(self, t):
        self.clock = max(self.clock, t)

    def cells(self, job):
        return job["nx"] * job["ny"]

    def required_bytes(self, job):
        return self.cells(job) * self.bpc

    def start(self, job):
        self.live[job["id"]] = self.required_bytes(job)
        self.max_live_bytes = max(self.max_live_bytes, sum(self.live.values()))
        return job

    def step(self, handles, steps):
        work = sum(self.cells(h) * n for h, n in zip(handles, steps))
        self.clock += self.overhead + work / (self.mlups * 1e6)
        self.calls.append([(h["id"], n) for h, n in zip(handles, steps)])

    def retire(self, h):
        return None

    def mark(self):
        return self.clock

    def wait(self, mark):
        pass

    def collect(self, h, pending):
        del self.live[h["id"]]
        return h["id"]

    def idle(self):
        pass

    def finish(self, h):
        return self.collect(h, self.retire(h))


class GpuBackend:
    """Jobs as lbm contexts on one GPU, memory from torch's allocator."""

    def __init__(self, device=0, keep_populations=False):
        import torch

        from . import lbm
        self.torch, self.lbm = torch, lbm
        self.dev = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.dev).cuda_stream
        self.keep = keep_populations
        # retired contexts: lbm_destroy waits for the shared stream, so they
        # are destroyed when the device has nothing queued
        self.retired = []

    def now(self):
        return time.perf_counter()

    def wait_until(self, t):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)

    def cells(self, job):
        return job["nx"] * job["ny"]

    def config(self, job):
        lbm = self.lbm
        nx, ny, U = job["nx"], job["ny"], job["ma"] * CS
        common = dict(lattice=lbm.LBM_D2Q9, shape=(nx, ny, 1), storage=job["storage"],
                      stream=self.stream, seed=job["seed"])
        if job["kind"] == "cylinder":
            D = max(ny // 10, 4)
            tau = 0.5 + 3.0 * U * D / 150.0
            W = max(nx // 8, 4)
            return lbm.make_config(tau=tau, ma=job["ma"], face_bc=(2, 2, 1, 1, 0, 0),
                                   sponge_width=(0, W, 0, 0, 0, 0), chi_max=0.2, rho_ref=1.0,
                                   u_ref=(U, 0.0, 0.0), **common)
        return lbm.make_config(tau=0.55, ma=job["ma"], **common)

    def required_bytes(self, job):
        return self.lbm.lbm_required_bytes(self.config(job))

    def fields(self, job):
        """Initial fields on the device: uniform flow U along x with a seeded
        1e-4 relative perturbation, and for pulse jobs a Gaussian density
        pulse (1e-3, sigma 8) at the centre; for cylinder jobs the SOLID disc
        of diameter ny/10 at (nx/5, ny/2) and the INLET column at x = 0."""
        t = self.torch
        nx, ny, U = job["nx"], job["ny"], job["ma"] * CS
        g = t.Generator(device=self.dev)
        g.manual_seed(job["seed"])
        y, x = t.meshgrid(t.arange(ny, device=self.dev, dtype=t.float64),
                          t.arange(nx, device=self.dev, dtype=t.float64), indexing="ij")
        u = t.zeros(3, ny * nx, dtype=t.float64, device=self.dev)
        u[0] = U
        u[:2] += 1e-4 * U * (2 * t.rand(2, ny * nx, generator=g, device=self.dev,
                                         dtype=t.float64) - 1)
        rho = t.ones(ny * nx, dtype=t.float64, device=self.dev)
        mask = None
        if job["kind"] == "pulse":
            r2 = (x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2
            rho += 1e-3 * t.exp(-r2 / (2 * 8.0 ** 2)).reshape(-1)
        else:
            D = max(ny // 10, 4)
            m = ((x - nx / 5.0) ** 2 + (y - ny / 2.0) ** 2 <= (D / 2.0) ** 2).to(t.uint8)
            m[:, 0] = 2
            mask = m.reshape(-1).contiguous()
        return rho, u, mask

    def start(self, job):
        lbm, t = self.lbm, self.torch
        cfg = self.config(job)
        need = lbm.lbm_required_bytes(cfg)
        mem = t.empty(need, dtype=t.uint8, device=self.dev)
        ctx = lbm.lbm_create(cfg)
        lbm.lbm_bind_memory(ctx, mem, need)
        rho, u, mask = self.fields(job)
        lbm.lbm_init(ctx, 0, rho, u, None, mask)
        return dict(ctx=ctx, mem=mem, keep=(rho, u, mask), job=job)

    def step(self, handles, steps):
        self.lbm.lbm_step_batch([h["ctx"] for h in handles], steps)

    def retire(self, h):
        """Enqueue the read-out of a job whose last quantum was just
        enqueued: its density (and, when kept, populations and initial
        fields) copied into pinned host memory behind that quantum."""
        lbm, t = self.lbm, self.torch
        n = self.cells(h["job"])

        def host(x):
            y = t.empty(x.shape, dtype=x.dtype, pin_memory=True)
            y.copy_(x, non_blocking=True)
            return y

        rho = t.empty(n, dtype=t.float64, device=self.dev)
        lbm.lbm_moments(h["ctx"], 0, rho, None)
        out = dict(rho=host(rho))
        if self.keep:
            # final populations and the initial fields the job started
            # from, for checking a job's result
            pops = t.empty(9, n, dtype=t.float64, device=self.dev)
            lbm.lbm_get_populations(h["ctx"], 0, pops)
            out["pops"] = host(pops)
            r0, u0, m0 = h["keep"]
            out["init"] = (host(r0), host(u0), None if m0 is None else host(m0))
        return out

    def mark(self):
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.dev))
        return ev

    def wait(self, ev):
        ev.synchronize()

    def collect(self, h, pending):
        """Result of a retired job once its read-out has completed; its
        memory goes back to torch's allocator (stream-ordered reuse) and its
        context is destroyed at the next idle point."""
        job = h["job"]
        out = dict(id=job["id"], rho=pending["rho"], rho_mean=float(pending["rho"].mean()),
                   pops=pending.get("pops"))
        if "init" in pending:
            out["init"] = tuple(None if x is None else x.numpy() for x in pending["init"])
        self.retired.append(h["ctx"])
        h["ctx"] = None
        del h["mem"], h["keep"]
        return out

    def idle(self):
        for ctx in self.retired:
            self.lbm.lbm_destroy(ctx)
        self.retired.clear()

    def finish(self, h):
        """Read out, wait and destroy one job (outside the serving loop)."""
        pending = self.retire(h)
        ev = self.mark()
        self.wait(ev)
        out = self.collect(h, pending)
        self.idle()
        return out
