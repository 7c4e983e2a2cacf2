"""Scheduling logic of the scan server on the CPU: a fake backend with a
mock clock (a simulated device that runs one chunk of steps per job after
another, all jobs in parallel), and the FP64 oracle behind the same backend
interface for the alone-vs-in-the-mix check."""
import numpy as np
import pytest

from paper_1912_04674_amd.serve import (ArenaAllocator, ScanServer, latency_stats, ALIGN, DONE, FAILED,
                                        CANCELLED, QUEUED, RUNNING)
from inputs import C1, scaled


class MockClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeBackend:
    """Each job costs `cost` seconds per step per million cells; chunks of a
    job complete one after another; a job may be told to fail at a step."""

    def __init__(self, clock, budget, cost=1e-3, fail_at=None, bad=None):
        self.clock, self.budget, self.cost = clock, budget, cost
        self.fail_at = fail_at or {}
        self.bad = bad or set()
        self.live = {}
        self.peak = 0

    def footprint(self, cfg):
        if cfg["name"] in self.bad:
            raise ValueError("invalid parameters")
        return cfg["nx"] * cfg["nr"] * 100

    def start(self, job, offset):
        h = {"job": job, "offset": offset, "end": self.clock(), "steps": []}
        self.live[job.id] = h
        used = sum(x["job"].footprint for x in self.live.values())
        assert used <= self.budget
        self.peak = max(self.peak, used)
        return h

    def issue(self, h, k):
        j = h["job"]
        first = len(h["steps"])
        if j.cfg["name"] in self.fail_at and first + k > self.fail_at[j.cfg["name"]]:
            raise RuntimeError("device error")
        h["steps"].extend(range(first, first + k))
        h["end"] = max(h["end"], self.clock()) + k * self.cost * j.cfg["nx"] * j.cfg["nr"] / 1e6
        return h["end"]

    def done(self, token):
        return self.clock() >= token

    def result(self, h):
        return {"steps": list(h["steps"]), "name": h["job"].cfg["name"]}

    def release(self, h):
        del self.live[h["job"].id]


def _jobs(n, rng, grids=((512, 64), (1024, 128), (2048, 256))):
    out = []
    for k in range(n):
        nx, nr = grids[int(rng.integers(0, len(grids)))]
        out.append(dict(name=f"j{k}", nx=nx, nr=nr, steps=int(rng.integers(50, 300))))
    return out


def test_allocator_first_fit_and_coalescing():
    a = ArenaAllocator(10 * ALIGN)
    x = a.alloc(1)
    y = a.alloc(ALIGN + 1)
    z = a.alloc(3 * ALIGN)
    assert (x, y, z) == (0, ALIGN, 3 * ALIGN)
    assert a.alloc(5 * ALIGN) is None and a.largest_free() == 4 * ALIGN
    a.release(y)
    assert a.alloc(2 * ALIGN) == ALIGN  # first fit reuses the hole
    a.release(x)
    a.release(ALIGN)
    a.release(z)
    assert a.free == [(0, 10 * ALIGN)] and a.bytes_free() == 10 * ALIGN


def test_allocator_random_against_interval_model():
    rng = np.random.default_rng(5)
    a = ArenaAllocator(64 * ALIGN)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off = list(live)[int(rng.integers(0, len(live)))]
            a.release(off)
            del live[off]
        else:
            n = int(rng.integers(1, 9 * ALIGN))
            off = a.alloc(n)
            need = -(-n // ALIGN) * ALIGN
            # first fit: the lowest aligned offset where `need` bytes are free
            occ = np.zeros(64, bool)
            for o, m in live.items():
                occ[o // ALIGN:(o + m) // ALIGN] = True
            want = None
            for s in range(0, 64 - need // ALIGN + 1):
                if not occ[s:s + need // ALIGN].any():
                    want = s * ALIGN
                    break
            assert off == want
            if off is not None:
                live[off] = need
    assert a.bytes_free() == 64 * ALIGN - sum(live.values())


def test_trace_all_jobs_done_within_budget():
    clk = MockClock()
    rng = np.random.default_rng(1)
    cfgs = _jobs(40, rng)
    arrivals = np.cumsum(rng.exponential(0.25, size=len(cfgs)))
    budget = 2048 * 256 * 100 * 2 + 1024 * 128 * 100  # two big jobs and a medium one at most
    be = FakeBackend(clk, budget)
    srv = ScanServer(be, budget_bytes=budget, max_slots=8, chunk=25, clock=clk)
    jobs = srv.run_trace(cfgs, arrivals, sleep=clk.sleep)
    assert all(j.status == DONE for j in jobs)
    for j, c in zip(jobs, cfgs):
        assert j.result["name"] == c["name"]
        assert j.result["steps"] == list(range(c["steps"]))  # every step once, in order
        assert j.admit >= j.arrival and j.finish >= j.admit
        assert j.latency >= c["steps"] * be.cost * c["nx"] * c["nr"] / 1e6 - 1e-9
    assert be.peak <= budget and be.live == {}
    assert srv.alloc.bytes_free() == srv.alloc.size
    st = latency_stats(jobs)
    assert st["n"] == 40 and st["p50"] <= st["p99"] == st["max"]


def test_jobs_overlap_when_they_fit():
    """Continuous batching: a job arriving while another runs starts at once."""
    clk = MockClock()
    be = FakeBackend(clk, 10**9)
    srv = ScanServer(be, budget_bytes=10**9, clock=clk)
    cfgs = [dict(name="a", nx=2048, nr=256, steps=300), dict(name="b", nx=512, nr=64, steps=300)]
    jobs = srv.run_trace(cfgs, [0.0, 0.05], sleep=clk.sleep)
    a, b = jobs
    assert b.admit - b.arrival < 1e-3 and b.admit < a.finish
    assert b.finish < a.finish  # the small job does not wait for the big one


def test_head_of_line_bypass_is_bounded():
    clk = MockClock()
    budget = 2048 * 256 * 100
    be = FakeBackend(clk, budget)
    srv = ScanServer(be, budget_bytes=budget, max_bypass=2, clock=clk)
    small = dict(name="s0", nx=512, nr=64, steps=100)
    srv.submit(small)
    srv.pump()  # s0 running: the big job cannot fit until it ends
    big = srv.submit(dict(name="big", nx=2048, nr=256, steps=10))
    later = [srv.submit(dict(name=f"s{k}", nx=512, nr=64, steps=100)) for k in range(1, 6)]
    srv.pump()
    st = [srv.jobs[i].status for i in later]
    assert st[:2] == [RUNNING, RUNNING] and all(s == QUEUED for s in st[2:])
    assert srv.jobs[big].status == QUEUED and srv.jobs[big].bypassed == 2
    while not srv.idle():
        srv.pump()
        clk.sleep(1e-3)
    order = sorted(srv.jobs.values(), key=lambda j: j.admit)
    names = [j.cfg["name"] for j in order]
    assert names.index("big") < names.index("s3")  # the head ran before the later jobs


def test_failures_and_cancellation_free_their_memory():
    clk = MockClock()
    budget = 10**9
    be = FakeBackend(clk, budget, fail_at={"f": 60}, bad={"bad"})
    srv = ScanServer(be, budget_bytes=budget, chunk=25, clock=clk)
    ids = {n: srv.submit(dict(name=n, nx=512, nr=64, steps=200)) for n in ("ok1", "f", "bad", "c1", "ok2")}
    assert srv.jobs[ids["bad"]].status == FAILED  # rejected at submission
    srv.pump()
    srv.cancel(ids["c1"])
    assert srv.jobs[ids["c1"]].status == CANCELLED
    while not srv.idle():
        srv.pump()
        clk.sleep(1e-3)
    assert srv.jobs[ids["f"]].status == FAILED and "device error" in srv.jobs[ids["f"]].error
    assert srv.jobs[ids["ok1"]].status == DONE and srv.jobs[ids["ok2"]].status == DONE
    assert srv.jobs[ids["ok2"]].result["steps"] == list(range(200))
    assert be.live == {} and srv.alloc.bytes_free() == srv.alloc.size


def test_oversized_job_is_rejected():
    clk = MockClock()
    be = FakeBackend(clk, 1000)
    srv = ScanServer(be, budget_bytes=100 * ALIGN, clock=clk)
    j = srv.submit(dict(name="huge", nx=2048, nr=256, steps=5))
    assert srv.jobs[j].status == FAILED and srv.idle()


# ------------------------------------------------ oracle behind the server --
class OracleBackend:
    """The FP64 oracle as a backend: steps run at issue time."""

    def __init__(self, oracle_mod):
        self.O = oracle_mod
        self.budget = 1 << 40

    def footprint(self, cfg):
        return cfg["nx"] * cfg["nr"] * 1000

    def start(self, job, offset):
        return self.O.OracleSim(job.cfg)

    def issue(self, sim, k):
        sim.step(k)
        return True

    def done(self, token):
        return True

    def result(self, sim):
        return {"diag": sim.diagnostics(), "ex": sim.get_field("ex"), "env": sim.get_field("env")}

    def release(self, sim):
        pass


def test_oracle_jobs_same_alone_and_in_the_mix(oracle_mod):
    base = scaled(C1, nx=48, nr=12, x_c=19.2, x_f=19.2, w0=8.0, tau=10.0, moving_window=1)
    cfgs = [scaled(base, a0=a0, n0=n0, seed=191204800 + k) for k, (a0, n0) in enumerate(((0.5, 0.002), (1.5, 0.003), (2.5, 0.001)))]
    srv = ScanServer(OracleBackend(oracle_mod), chunk=7, max_slots=2)
    jobs = srv.run_trace(cfgs, [0.0, 0.0, 0.0], steps=30, sleep=lambda dt: None)
    for c, j in zip(cfgs, jobs):
        assert j.status == DONE
        alone = oracle_mod.OracleSim(c)
        alone.step(30)
        np.testing.assert_array_equal(j.result["ex"], alone.get_field("ex"))
        np.testing.assert_array_equal(j.result["env"], alone.get_field("env"))
