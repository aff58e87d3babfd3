"""Served continuous batching of lattice jobs on one GPU.

A request loop keeps the populations of every admitted job resident in one
device arena.  Queued jobs are admitted first in, first out as soon as the
arena has room for their exact footprint (``dsm_required_bytes``); resident
jobs advance together, a quantum of steps at a time, through the batched
step of libdsm.so (one batch per population storage), so the work of jobs
that arrived at different times overlaps in the same launches.  A job that
arrives while others run joins at the next quantum boundary; a quantum never
runs past the step count any resident job asked for, so each job leaves at
exactly its own step and its result is the one it would have alone.

A job that fails (its set-up is rejected, or its lattice goes non-finite)
is retired with its error, its arena slot freed, while the others go on:
the lattices of a batch are independent, so its failure changes no other
job's result.

Set-up and result readout go through the executor's ``start_async`` and
``finish_async``: the GPU executor runs them on a worker thread and a stream
of their own while the resident jobs' quantum runs, so the GPU does not idle
through them; a job joins the batch at the first quantum boundary after its
set-up has finished, and its arena slot is freed once its result has been
read.  The timing-model executor completes both at once.

The scheduling logic (``Arena``, ``Server``, ``run_stream``) is plain host
code; device work goes through an executor: ``GpuExecutor`` drives the C ABI,
``ModelExecutor`` replaces it with a timing model for host-only tests.
"""
from __future__ import annotations

import collections
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

ALIGN = 256


class Arena:
    """First-fit allocator over the byte range [0, capacity): blocks are
    rounded up to 256 bytes, free neighbours merge."""

    def __init__(self, capacity: int, align: int = ALIGN):
        self.align = align
        self.capacity = capacity // align * align
        self.free_list = [(0, self.capacity)] if self.capacity else []  # (offset, size), by offset
        self.blocks = {}  # offset -> size
        self.peak = 0

    @property
    def used(self) -> int:
        return sum(self.blocks.values())

    @property
    def largest_free(self) -> int:
        return max((s for _, s in self.free_list), default=0)

    def round(self, nbytes: int) -> int:
        return max(self.align, -(-int(nbytes) // self.align) * self.align)

    def alloc(self, nbytes: int):
        size = self.round(nbytes)
        for k, (off, s) in enumerate(self.free_list):
            if s >= size:
                if s == size:
                    del self.free_list[k]
                else:
                    self.free_list[k] = (off + size, s - size)
                self.blocks[off] = size
                self.peak = max(self.peak, self.used)
                return off
        return None

    def free(self, off: int):
        size = self.blocks.pop(off)
        fl = self.free_list
        k = 0
        while k < len(fl) and fl[k][0] < off:
            k += 1
        fl.insert(k, (off, size))
        if k + 1 < len(fl) and fl[k][0] + fl[k][1] == fl[k + 1][0]:
            fl[k] = (fl[k][0], fl[k][1] + fl[k + 1][1])
            del fl[k + 1]
        if k > 0 and fl[k - 1][0] + fl[k - 1][1] == fl[k][0]:
            fl[k - 1] = (fl[k - 1][0], fl[k - 1][1] + fl[k][1])
            del fl[k]


@dataclass
class Job:
    """One simulation request: a workload (geometry, parameters, initial
    liquid), the number of fluid steps to run, the population storage."""
    id: int
    workload: object
    steps: int
    storage: int = 0
    arrival: float = 0.0
    nbytes: int = 0
    offset: int | None = None
    done_steps: int = 0
    admitted: float | None = None
    finished: float | None = None
    result: dict | None = None
    error: str | None = None  # set when the job failed (result stays None)

    @property
    def nodes(self) -> int:
        return int(np.prod(self.workload.shape))

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """The request loop's state: queue, arena, resident jobs.  ``step``
    performs one round: admit what fits, rebuild the batches if the resident
    set changed, run one quantum, retire the jobs that reached their step
    count.  Times passed in are seconds on the caller's clock."""

    def __init__(self, executor, capacity: int, quantum: int = 50, table_fraction: float = 1.0 / 256):
        self.ex = executor
        tables = max(16 << 20, int(capacity * table_fraction)) // ALIGN * ALIGN
        if capacity <= tables:
            raise ValueError("capacity too small")
        self.arena = Arena(capacity - tables)
        self.tables = Arena(tables)
        self.table_blocks = {}
        self.quantum = int(quantum)
        self.queue = collections.deque()
        self.running = []
        self.setting_up = []  # (job, future of its set-up), in admission order
        self.finishing = []   # (job, future of (result, time read or None))
        self.done = []
        self.failed = []
        self.changed = False
        self.rounds = 0
        self.steps_run = 0

    @property
    def busy(self) -> bool:
        return bool(self.queue or self.running or self.setting_up or self.finishing)

    def submit(self, job: Job, now: float):
        job.arrival = now
        job.nbytes = self.ex.job_bytes(job)
        if self.arena.round(job.nbytes) > self.arena.capacity:
            raise ValueError(f"job {job.id} needs {job.nbytes} bytes, more than the arena holds")
        if job.steps < 1:
            raise ValueError(f"job {job.id}: steps must be >= 1")
        self.queue.append(job)

    def _admit(self, now: float):
        while self.queue:
            job = self.queue[0]
            off = self.arena.alloc(job.nbytes)
            if off is None:
                break  # first in, first out: later jobs wait behind the head
            self.queue.popleft()
            job.offset = off
            job.admitted = now
            self.setting_up.append((job, self.ex.start_async(job, off)))

    def _join(self, now: float, wait: bool) -> bool:
        """Jobs whose set-up has finished join the resident set (in admission
        order); with ``wait``, blocks until the oldest set-up has finished.
        Returns whether any joined."""
        if wait and self.setting_up:
            _wait(self.setting_up[0][1])
        joined, keep = False, []
        for job, fut in self.setting_up:
            if not fut.done():
                keep.append((job, fut))
                continue
            try:
                job.done_steps = fut.result()
            except Exception as e:  # noqa: BLE001 (any set-up error fails this job only)
                self.arena.free(job.offset)
                job.offset = None
                self._retire_failed(job, f"{type(e).__name__}: {e}", now)
                continue
            self.running.append(job)
            joined = True
        self.setting_up = keep
        return joined

    def _collect(self, now: float, wait: bool) -> list:
        """Jobs whose result has been read: result, finish time, slot freed.
        With ``wait``, blocks until the oldest readout has finished."""
        if wait and self.finishing:
            _wait(self.finishing[0][1])
        out, keep = [], []
        for job, fut in self.finishing:
            if not fut.done():
                keep.append((job, fut))
                continue
            self.arena.free(job.offset)
            try:
                job.result, t_read = fut.result()
            except Exception as e:  # noqa: BLE001 (a failed readout fails this job only)
                self._retire_failed(job, f"{type(e).__name__}: {e}", now)
                continue
            job.finished = now if t_read is None else t_read
            self.done.append(job)
            out.append(job)
        self.finishing = keep
        return out

    def _retire_failed(self, job: Job, error: str, t: float):
        job.error = error
        job.finished = t
        self.failed.append(job)

    def _rebuild(self):
        for off in self.table_blocks.values():
            self.tables.free(off)
        self.table_blocks = {}
        while True:
            need = self.ex.table_bytes(self.running)
            blocks = {}
            ok = True
            for key, nbytes in need.items():
                off = self.tables.alloc(nbytes)
                if off is None:
                    ok = False
                    break
                blocks[key] = off
            if ok:
                self.table_blocks = blocks
                self.ex.rebuild(self.running, blocks)
                return
            for off in blocks.values():
                self.tables.free(off)
            # the tables of this resident set do not fit: send the newest
            # job back to the head of the queue
            job = self.running.pop()
            self.ex.drop(job)
            self.arena.free(job.offset)
            job.offset, job.admitted, job.done_steps = None, None, 0
            self.queue.appendleft(job)

    def step(self, now: float, clock=None) -> list:
        """One round; returns the jobs whose results were read in it."""
        finished = self._collect(now, wait=False)
        self._admit(now)
        # with nothing resident, wait for a set-up (else for a readout, which
        # frees arena room) rather than spin
        idle = not self.running
        if self._join(now, wait=idle):
            self.changed = True
        if not self.running and not self.setting_up:
            finished += self._collect(clock() if clock else now, wait=idle)
        if self.changed:
            self._rebuild()
            self.changed = False
        failed = {}
        if self.running:
            k = min(self.quantum, min(j.steps - j.done_steps for j in self.running))
            if k > 0:
                failed = self.ex.advance(k) or {}
                self.steps_run += k
                for j in self.running:
                    j.done_steps += k
        self.rounds += 1
        t = clock() if clock else now
        for j in [j for j in self.running if j.id in failed]:
            self.ex.drop(j)
            self.arena.free(j.offset)
            self.running.remove(j)
            self._retire_failed(j, failed[j.id], t)
            self.changed = True
        for j in [j for j in self.running if j.done_steps >= j.steps]:
            self.running.remove(j)
            self.finishing.append((j, self.ex.finish_async(j, clock)))
            self.changed = True
        return finished + self._collect(t, wait=False)


def _wait(fut):
    """Blocks until a future has finished (its outcome is read later)."""
    if not fut.done():
        try:
            fut.result()
        except Exception:  # noqa: BLE001 (handled where the result is read)
            pass


class _Done:
    """A future that has already finished (for executors without a worker)."""

    def __init__(self, fn, *args):
        try:
            self._value, self._error = fn(*args), None
        except Exception as e:  # noqa: BLE001 (re-raised by result())
            self._value, self._error = None, e

    def done(self) -> bool:
        return True

    def result(self):
        if self._error is not None:
            raise self._error
        return self._value


def run_stream(server: Server, jobs, arrivals, clock=time.perf_counter, sleep=time.sleep):
    """Feeds jobs to the server at their arrival times (seconds from the
    start) and runs rounds until every job has finished.  Returns the
    elapsed time."""
    pending = collections.deque(sorted(zip(arrivals, range(len(jobs))), key=lambda p: p[0]))
    t0 = clock()
    now = lambda: clock() - t0  # noqa: E731
    while pending or server.busy:
        t = now()
        while pending and pending[0][0] <= t:
            at, k = pending.popleft()
            server.submit(jobs[k], at)
        if not server.busy:
            sleep(max(0.0, pending[0][0] - t))
            continue
        server.step(t, now)
    return now()


def poisson_arrivals(count: int, rate: float, seed: int) -> list:
    """Arrival times (s) of a Poisson stream of the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return list(np.cumsum(rng.exponential(1.0 / rate, size=count)))


def report(jobs, elapsed: float) -> dict:
    """Latency and throughput over the jobs that finished; failed jobs are
    counted apart."""
    failed = [j for j in jobs if j.error is not None]
    jobs = [j for j in jobs if j.error is None]
    lat = np.array([j.latency for j in jobs])
    wait = np.array([j.admitted - j.arrival for j in jobs])
    work = sum(j.nodes * j.steps for j in jobs)
    return {
        "jobs": len(jobs),
        "failed_jobs": len(failed),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
        "max_latency_s": round(float(lat.max()), 4),
        "p50_queue_wait_s": round(float(np.percentile(wait, 50)), 4),
        "elapsed_s": round(elapsed, 3),
        "aggregate_mlups": round(work / elapsed / 1e6, 2),
    }


class ModelExecutor:
    """Stand-in for the GPU: footprints and step times from a model, results
    that record what was run.  Time advances on a virtual clock shared with
    the caller (``now``), one quantum taking sum(nodes) / rate seconds per
    step plus a fixed overhead."""

    def __init__(self, rate: float = 1e10, overhead: float = 1e-4, bytes_per_node: int = 400,
                 fail_start=(), fail_at=None):
        self.rate, self.overhead, self.bpn = rate, overhead, bytes_per_node
        self.t = 0.0
        self.resident = {}
        self.members = set()  # job ids of the last rebuild: the ones a quantum steps
        self.log = []
        self.fail_start = set(fail_start)   # job ids whose set-up is rejected
        self.fail_at = dict(fail_at or {})  # job id -> step at which it goes non-finite

    def now(self) -> float:
        return self.t

    def sleep(self, dt: float):
        self.t += dt

    def job_bytes(self, job) -> int:
        return job.nodes * self.bpn + 4096

    def start_async(self, job, offset):
        return _Done(self.start, job, offset)

    def finish_async(self, job, clock=None):
        return _Done(lambda: (self.finish(job), None))

    def start(self, job, offset) -> int:
        if job.id in self.fail_start:
            raise RuntimeError(f"set-up of job {job.id} rejected")
        self.resident[job.id] = {"offset": offset, "steps": 1, "nodes": job.nodes}
        self.t += self.overhead
        return 1

    def table_bytes(self, running) -> dict:
        out = {}
        for j in running:
            out[j.storage] = out.get(j.storage, 0) + j.nodes // 8 + 1024
        return out

    def rebuild(self, running, blocks):
        self.members = {j.id for j in running}
        self.log.append(("rebuild", sorted(self.members)))

    def advance(self, n: int) -> dict:
        failed = {}
        stepped = {jid: r for jid, r in self.resident.items() if jid in self.members}
        for jid, r in stepped.items():
            r["steps"] += n
            if jid in self.fail_at and r["steps"] >= self.fail_at[jid]:
                failed[jid] = "non-finite values"
        nodes = sum(r["nodes"] for r in stepped.values())
        self.log.append(("advance", n, sorted(stepped)))
        self.t += self.overhead + n * nodes / self.rate
        return failed

    def finish(self, job) -> dict:
        r = self.resident.pop(job.id)
        return {"steps": r["steps"], "offset": r["offset"]}

    def drop(self, job):
        self.resident.pop(job.id)


class GpuExecutor:
    """Device side of the server: one torch buffer as the arena, one
    Simulation per resident job carved from it, one Batch per storage.

    Set-up and readout run on one worker thread, with the jobs' handles on
    a stream of their own; the batches step on another stream from the
    request loop's thread.  A set-up ends by synchronising its stream (the
    job's state is complete before any batch reads it), a readout starts
    after the quantum that finished the job has been synchronised, and a
    job's handle is used by one thread at a time."""

    def __init__(self, capacity: int, device="cuda:0"):
        import torch

        from . import dsm

        self.dsm = dsm
        dsm.load()  # raises if the HIP library is missing: there is no fallback
        self.torch = torch
        self.device = torch.device(device)
        self.buffer = torch.empty(capacity + 2 * ALIGN, dtype=torch.uint8, device=self.device)
        self.base = (self.buffer.data_ptr() + ALIGN - 1) // ALIGN * ALIGN
        self.capacity = capacity
        # default-priority streams, neither of them the null stream, so that
        # set-up and readout overlap the batched steps
        self.job_stream = torch.cuda.Stream(self.device)
        self.batch_stream = torch.cuda.Stream(self.device)
        torch.cuda.synchronize(self.device)  # the arena's allocation is complete
        self.worker = ThreadPoolExecutor(max_workers=1)
        self.sims = {}
        self.batches = {}
        self.members = {}  # batch key -> job ids, in member order
        self.table_base = None

    def start_async(self, job, offset):
        return self.worker.submit(self.start, job, offset)

    def finish_async(self, job, clock=None):
        def read():
            out = self.finish(job)
            return out, (clock() if clock else None)
        return self.worker.submit(read)

    def close(self):
        self.worker.shutdown(wait=True)

    def set_table_base(self, base: int):
        self.table_base = base

    def _params(self, job):
        w = job.workload
        return self.dsm.make_params(w.dim, w.shape, w.kappa, w.alpha, w.tau, w.mobility, w.gravity,
                                    storage=job.storage, rho=w.rho, tau_gas=w.tau_gas or 0.0)

    def job_bytes(self, job) -> int:
        return self.dsm.dsm_required_bytes(self._params(job))

    def start(self, job, offset) -> int:
        from . import workloads as W

        w = job.workload
        self.torch.cuda.set_device(self.device)  # this thread's current device
        sim = self.dsm.Simulation(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                                  gravity=w.gravity, storage=job.storage, device=self.device,
                                  stream=self.job_stream, dev_ptr=self.base + offset, rho=w.rho,
                                  tau_gas=w.tau_gas or 0.0)
        try:
            # the library rounds the FP64 fields to FP32 itself
            sim.set_solid_field(W.flat(w.C1))
            sim.set_liquid(W.flat(w.C2))
            sim.step(1)  # the first step reads at-node populations; later steps run batched
            self.job_stream.synchronize()
        except Exception:
            sim.close()
            raise
        self.sims[job.id] = sim
        return 1

    def table_bytes(self, running) -> dict:
        groups = {}
        for j in running:
            groups.setdefault(j.storage, []).append(self.sims[j.id].handle)
        return {k: self.dsm.dsm_batch_required_bytes(v) for k, v in groups.items()}

    def rebuild(self, running, blocks):
        for b in self.batches.values():
            b.close()
        self.batches = {}
        self.members = {}
        for j in running:
            self.members.setdefault(j.storage, []).append(j.id)
        for key, ids in self.members.items():
            b = self.dsm.Batch([self.sims[i] for i in ids], device=self.device, stream=self.batch_stream,
                               dev_ptr=self.table_base + blocks[key])
            b.tune()
            self.batches[key] = b

    def _unstable(self, jid) -> bool:
        d = self.sims[jid].diagnostics()
        return d["nonfinite_nodes"] > 0 or not np.isfinite(d["max_speed"]) or not np.all(np.isfinite(d["mass"]))

    def advance(self, n: int) -> dict:
        """n steps of every batch; returns {job id: error} of the jobs whose
        lattice went non-finite (the batch's check names the failure, each
        member's FP64 diagnostics say which; the others advanced normally)."""
        failed = {}
        for key, b in self.batches.items():
            try:
                b.step(n)
            except self.dsm.DsmError as e:
                if e.code != self.dsm.DSM_EUNSTABLE:
                    raise
                bad = [i for i in self.members[key] if self._unstable(i)] or list(self.members[key])
                for i in bad:
                    failed[i] = f"DSM_EUNSTABLE: {e}"
        return failed

    def finish(self, job) -> dict:
        self.torch.cuda.set_device(self.device)  # this thread's current device
        sim = self.sims.pop(job.id)
        # C2 alone (one plane copied), then one FP64 reduction for the masses
        # and the free energy
        d = sim.diagnostics()
        out = {"C2": sim.fields(("C2",))["C2"], "mass": d["mass"], "free_energy": d["free_energy"],
               "steps": sim.steps}
        sim.close()
        return out

    def drop(self, job):
        self.sims.pop(job.id).close()


def make_gpu_server(capacity: int, quantum: int = 50, device="cuda:0") -> Server:
    """A server whose arena and batch tables live in one device buffer of
    ``capacity`` bytes."""
    ex = GpuExecutor(capacity, device)
    srv = Server(ex, capacity, quantum)
    ex.set_table_base(ex.base + srv.arena.capacity)
    return srv
