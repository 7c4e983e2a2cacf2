"""Continuous-batching server for parametric-scan jobs (many small envelope
PIC runs resident on one GPU at once).

A job is a parameter block (a0, density, waist, grid size, ...) and a step
count.  Jobs arrive at any time; the server admits them in arrival order as
soon as their device footprint fits in a fixed arena (first fit, 256-byte
aligned) and a slot is free, steps every admitted job on its own HIP stream
so that the kernels of different jobs overlap on the device, and retires a
job when its last step has completed and its result has reached the host.
Memory is taken once, up front: serving allocates nothing on the device.

The step work itself runs in libenvpic (the HIP kernels); this module is host
orchestration only.  The device work is hidden behind a small backend
interface (`GpuBackend` here); tests plug in a CPU backend with a mock
clock to check the scheduling logic.
"""
import time
from dataclasses import dataclass, field

ALIGN = 256

QUEUED, RUNNING, DONE, FAILED, CANCELLED = "queued", "running", "done", "failed", "cancelled"


class ArenaAllocator:
    """First-fit allocator of [0, size) in ALIGN-byte units (host bookkeeping
    of one device arena).  Free blocks are coalesced on release."""

    def __init__(self, size):
        self.size = int(size) // ALIGN * ALIGN
        self.free = [(0, self.size)]  # sorted (offset, length)
        self.used = {}

    def alloc(self, nbytes):
        n = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for k, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + n, ln - n)
                self.used[off] = n
                return off
        return None

    def release(self, off):
        n = self.used.pop(off)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    def bytes_free(self):
        return sum(ln for _, ln in self.free)

    def largest_free(self):
        return max((ln for _, ln in self.free), default=0)


@dataclass
class Job:
    id: int
    cfg: dict
    steps: int
    arrival: float
    status: str = QUEUED
    footprint: int = 0
    offset: int = -1
    admit: float = None
    finish: float = None
    issued: int = 0
    bypassed: int = 0
    pending: list = field(default_factory=list)
    handle: object = None
    result: dict = None
    error: str = None
    extra: dict = field(default_factory=dict)

    @property
    def latency(self):
        return None if self.finish is None else self.finish - self.arrival


class GpuBackend:
    """Jobs as libenvpic simulations inside one pre-allocated device arena,
    each on a pooled HIP stream (default priority).

    With `graph_min_jobs` or more jobs resident, a job's chunk of steps is
    issued as one HIP graph (envpic_set_graph): issuing small jobs' kernels
    one by one then keeps the host busier than the device.  With fewer jobs
    the kernels are launched directly, which runs a lone job faster."""

    def __init__(self, budget_bytes, precision=0, lineout=True, full=False, graph_min_jobs=4,
                 beam_query=(1e-3, 20.0, 256)):
        import torch
        from . import envpic as E
        self.E, self.torch = E, torch
        E.lib()
        self.precision = precision
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device="cuda")
        self.budget = int(budget_bytes)
        self.lineout, self.full = lineout, full
        # (e_lo, e_hi, nbins) of the injected-beam parameters returned with
        # each result (a job's cfg may give its own as "beam_query"); None: off
        self.beam_query = beam_query
        self.graph_min_jobs = graph_min_jobs
        self._streams = []
        self._live = 0

    def footprint(self, cfg):
        return self.E.footprint(cfg, self.precision)

    def start(self, job, offset):
        torch = self.torch
        st = self._streams.pop() if self._streams else torch.cuda.Stream()
        view = self.arena[offset:offset + job.footprint]
        sim = self.E.Sim(job.cfg, self.precision, arena=view, stream=st)
        self._live += 1
        return {"sim": sim, "stream": st, "view": view, "graph": 0,
                "beam_query": job.cfg.get("beam_query", self.beam_query)}

    def issue(self, h, k):
        """Queue k steps on the job's stream; returns a completion token."""
        g = k if self.graph_min_jobs and self._live >= self.graph_min_jobs else 0
        if g != h["graph"]:
            h["sim"].set_graph(g)
            h["graph"] = g
        h["sim"].step(k)
        ev = self.torch.cuda.Event()
        ev.record(h["stream"])
        return ev

    def done(self, token):
        return token.query()

    def result(self, h):
        sim = h["sim"]
        out = {"diag": sim.diagnostics()}
        if h["beam_query"] is not None:
            out["beam"] = sim.beam(*h["beam_query"])
        if self.lineout:
            out["ex_axis"] = sim.get_field("ex")[:, 0].copy()
        if self.full:  # the whole final state (for checks)
            out["fields"] = {n: sim.get_field(n) for n in ("env", "chi", "ex", "er", "bt")}
            out["particles"] = sim.get_particles()
        return out

    def release(self, h):
        h["stream"].synchronize()
        h["sim"].close()
        self._live -= 1
        self._streams.append(h["stream"])


class ScanServer:
    """Continuous batching over a backend.

    submit() queues a job; pump() retires finished jobs, admits queued jobs
    that fit (arrival order; a later job may pass a head that does not fit,
    but a head passed `max_bypass` times blocks further admissions until it
    fits), and issues up to `chunk` more steps to every running job that has
    fewer than `depth` chunks in flight."""

    def __init__(self, backend, budget_bytes=None, max_slots=32, chunk=25, depth=2, max_bypass=8,
                 clock=time.perf_counter):
        self.backend = backend
        self.alloc = ArenaAllocator(budget_bytes if budget_bytes is not None else backend.budget)
        self.max_slots, self.chunk, self.depth, self.max_bypass = max_slots, chunk, depth, max_bypass
        self.clock = clock
        self.jobs = {}
        self.queue = []
        self.running = []
        self._next = 0

    # ---------------------------------------------------------------- API --
    def submit(self, cfg, steps=None, arrival=None):
        j = Job(self._next, dict(cfg), int(steps if steps is not None else cfg.get("steps", 1)),
                self.clock() if arrival is None else arrival)
        self._next += 1
        try:
            j.footprint = int(self.backend.footprint(j.cfg))
        except Exception as e:  # invalid parameters: rejected at submission
            j.status, j.error, j.finish = FAILED, str(e), j.arrival
            self.jobs[j.id] = j
            return j.id
        if j.footprint > self.alloc.size:
            j.status, j.error, j.finish = FAILED, "footprint exceeds the arena", j.arrival
        else:
            self.queue.append(j)
        self.jobs[j.id] = j
        return j.id

    def cancel(self, job_id):
        j = self.jobs[job_id]
        if j.status == QUEUED:
            self.queue.remove(j)
            j.status, j.finish = CANCELLED, self.clock()
        elif j.status == RUNNING:
            self._retire(j, CANCELLED)

    def idle(self):
        return not self.queue and not self.running

    def pump(self):
        """One scheduling round; returns the ids of jobs that ended in it."""
        ended = []
        for j in list(self.running):
            while j.pending and self.backend.done(j.pending[0]):
                j.pending.pop(0)
            if j.issued >= j.steps and not j.pending:
                try:
                    j.result = self.backend.result(j.handle)
                    self._retire(j, DONE)
                except Exception as e:
                    j.error = str(e)
                    self._retire(j, FAILED)
                ended.append(j.id)
        self._admit(ended)
        for j in list(self.running):
            if j.issued < j.steps and len(j.pending) < self.depth:
                k = min(self.chunk, j.steps - j.issued)
                try:
                    j.pending.append(self.backend.issue(j.handle, k))
                    j.issued += k
                except Exception as e:
                    j.error = str(e)
                    self._retire(j, FAILED)
                    ended.append(j.id)
        return ended

    def run_trace(self, cfgs, arrivals, steps=None, sleep=time.sleep, poll=0.0005, timeout=None):
        """Submit cfgs[k] at arrivals[k] (seconds after the start) and serve
        until every job has ended.  Returns the jobs in submission order."""
        t0 = self.clock()
        order = sorted(range(len(cfgs)), key=lambda k: arrivals[k])
        nxt, ids = 0, {}
        while nxt < len(order) or not self.idle():
            now = self.clock() - t0
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                k = order[nxt]
                ids[k] = self.submit(cfgs[k], steps, arrival=t0 + arrivals[k])
                nxt += 1
            self.pump()
            if timeout is not None and now > timeout:
                raise TimeoutError("trace did not finish")
            if nxt < len(order) and self.idle():
                sleep(max(0.0, arrivals[order[nxt]] - (self.clock() - t0)))
            elif not self.idle():
                sleep(poll)
        return [self.jobs[ids[k]] for k in range(len(cfgs))]

    # ------------------------------------------------------------ helpers --
    def _admit(self, ended):
        for j in list(self.queue):
            if len(self.running) >= self.max_slots:
                break
            head = self.queue[0]
            if j is not head and head.bypassed >= self.max_bypass:
                break  # the head has waited long enough: nobody else passes it
            off = self.alloc.alloc(j.footprint)
            if off is None:
                continue
            if j is not head:
                head.bypassed += 1
            self.queue.remove(j)
            j.offset, j.admit = off, self.clock()
            try:
                j.handle = self.backend.start(j, off)
                j.status = RUNNING
                self.running.append(j)
            except Exception as e:
                j.error = str(e)
                self._retire(j, FAILED)
                ended.append(j.id)

    def _retire(self, j, status):
        j.pending = []
        if j.handle is not None:
            try:
                self.backend.release(j.handle)
            finally:
                j.handle = None
        if j.offset >= 0:
            self.alloc.release(j.offset)
            j.offset = -1
        if j in self.running:
            self.running.remove(j)
        j.status = status
        j.finish = self.clock()


def latency_stats(jobs):
    """Nearest-rank p50 / p99 of the completed jobs' latencies (seconds)."""
    lat = sorted(j.latency for j in jobs if j.status == DONE)
    if not lat:
        return {"p50": None, "p99": None, "n": 0}

    def rank(q):
        k = max(1, int(-(-q * len(lat) // 1)))  # ceil(q n)
        return lat[min(len(lat), k) - 1]
    return {"p50": rank(0.50), "p99": rank(0.99), "n": len(lat), "max": lat[-1], "mean": sum(lat) / len(lat)}
