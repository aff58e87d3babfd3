"""Host logic of the served form, without a GPU: the arena allocator, and
the request loop driven by a timing-model executor (admission by footprint,
first in first out, joining at quantum boundaries, exact step counts,
retirement, latency report)."""
import threading
import time
import types
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2504_19941_amd import serve as S


def test_arena_first_fit_alignment_and_merging():
    a = S.Arena(10 * 256)
    x = a.alloc(1)
    y = a.alloc(300)
    z = a.alloc(256)
    assert (x, y, z) == (0, 256, 768)
    assert a.used == 4 * 256
    assert a.alloc(7 * 256) is None  # only 6 blocks left
    a.free(y)
    assert a.alloc(2 * 256) == 256  # first fit reuses the hole
    a.free(256)
    a.free(x)
    a.free(z)
    assert a.free_list == [(0, 10 * 256)] and a.used == 0
    assert a.peak == 4 * 256


def test_arena_random_sequence_never_overlaps():
    rng = np.random.default_rng(3)
    cap = 4096 * 256
    a = S.Arena(cap)
    owner = np.zeros(cap // 256, dtype=np.int64)  # brute-force occupancy map
    live = {}
    for it in range(3000):
        if live and rng.uniform() < 0.45:
            off = list(live)[rng.integers(len(live))]
            size = live.pop(off)
            assert np.all(owner[off // 256:(off + size) // 256] == off + 1)
            owner[off // 256:(off + size) // 256] = 0
            a.free(off)
        else:
            n = int(rng.integers(1, 200 * 256))
            off = a.alloc(n)
            need = a.round(n) // 256
            if off is None:
                # first fit fails only if no free run is large enough
                assert a.largest_free < need * 256
                continue
            assert off % 256 == 0
            assert np.all(owner[off // 256:off // 256 + need] == 0)
            owner[off // 256:off // 256 + need] = off + 1
            live[off] = need * 256
        assert a.used == sum(live.values()) <= cap
        # free list: sorted, disjoint, merged, and the complement of the blocks
        fl = a.free_list
        assert all(fl[k][0] + fl[k][1] < fl[k + 1][0] for k in range(len(fl) - 1))
        assert sum(s for _, s in fl) + a.used == cap


def job(jid, shape, steps, storage=0):
    w = types.SimpleNamespace(shape=shape)
    return S.Job(jid, w, steps, storage)


def test_server_runs_every_job_exactly_and_within_budget():
    ex = S.ModelExecutor(rate=2e9, overhead=1e-4)
    cap = 256 << 20  # 240 MiB of arena: a handful of these jobs at once
    srv = S.Server(ex, cap, quantum=20)
    rng = np.random.default_rng(11)
    jobs = [job(k, (int(rng.integers(16, 60)),) * 3, int(rng.integers(1, 300)), storage=k % 2) for k in range(40)]
    arrivals = S.poisson_arrivals(len(jobs), rate=200.0, seed=2)
    peak = [0]
    orig = srv.step

    def step(now, clock=None):
        out = orig(now, clock)
        peak[0] = max(peak[0], srv.arena.used)
        assert srv.arena.used <= srv.arena.capacity
        return out

    srv.step = step
    elapsed = S.run_stream(srv, jobs, arrivals, clock=ex.now, sleep=ex.sleep)
    assert len(srv.done) == len(jobs)
    for j in jobs:
        assert j.result["steps"] == j.steps  # never past, never short
        assert j.finished >= j.admitted >= j.arrival
    # first in, first out
    order = sorted(jobs, key=lambda j: j.arrival)
    adm = [j.admitted for j in order]
    assert adm == sorted(adm)
    # the budget was the binding constraint at some point (jobs queued)
    assert any(j.admitted > j.arrival for j in jobs)
    assert peak[0] <= srv.arena.capacity
    rep = S.report(jobs, elapsed)
    assert rep["jobs"] == 40 and rep["p99_latency_s"] >= rep["p50_latency_s"] > 0


def test_jobs_join_running_ones_at_quantum_boundaries():
    ex = S.ModelExecutor(rate=1e8, overhead=0.0)
    srv = S.Server(ex, 1 << 30, quantum=10)
    a, b = job(0, (32, 32, 32), 95), job(1, (20, 20, 20), 31)
    srv.submit(a, 0.0)
    srv.step(0.0)            # a admitted (1 step) and advanced 10
    srv.submit(b, 0.001)     # b arrives while a runs
    srv.step(0.001)          # b joins: the quantum covers both
    adv = [e for e in ex.log if e[0] == "advance"]
    assert adv[0][2] == [0] and adv[1][2] == [0, 1]
    while srv.busy:
        srv.step(1.0)
    assert a.result["steps"] == 95 and b.result["steps"] == 31
    # a quantum never carried b past its step count
    assert all(e[1] <= 10 for e in adv)


def test_oversized_job_is_rejected_and_one_step_jobs_finish():
    ex = S.ModelExecutor()
    srv = S.Server(ex, 32 << 20, quantum=8)
    with pytest.raises(ValueError):
        srv.submit(job(0, (300, 300, 300), 10), 0.0)
    with pytest.raises(ValueError):
        srv.submit(job(1, (8, 8, 8), 0), 0.0)
    one = job(2, (8, 8, 8), 1)
    srv.submit(one, 0.0)
    srv.step(0.0)
    assert one.result["steps"] == 1 and not srv.busy


def test_batch_tables_that_do_not_fit_send_the_newest_job_back():
    class Tight(S.ModelExecutor):
        def table_bytes(self, running):
            # every resident job needs a quarter of the table region
            return {0: len(running) * (4 << 20)}

    ex = Tight()
    srv = S.Server(ex, 1 << 30, quantum=5)  # table region: 16 MiB -> 4 jobs at once
    jobs = [job(k, (8, 8, 8), 12) for k in range(6)]
    for j in jobs:
        srv.submit(j, 0.0)
    srv.step(0.0)
    assert len(srv.running) == 4 and len(srv.queue) == 2
    assert [j.id for j in srv.queue] == [4, 5]
    while srv.busy:
        srv.step(1.0)
    assert all(j.result["steps"] == 12 for j in jobs)


def test_failed_jobs_are_retired_and_the_others_finish():
    """A job whose set-up is rejected and one whose lattice goes non-finite
    in the middle of a quantum are retired with their errors and their arena
    slots freed; every other job still runs exactly its steps, including the
    ones that shared the failing quanta and the ones queued behind."""
    ex = S.ModelExecutor(rate=1e9, overhead=1e-4, fail_start={3}, fail_at={5: 37})
    srv = S.Server(ex, 100 << 20, quantum=10)  # room for three of these jobs at once
    jobs = [job(k, (40, 40, 40), 60 + 5 * k) for k in range(10)]
    arrivals = [0.0005 * k for k in range(10)]
    elapsed = S.run_stream(srv, jobs, arrivals, clock=ex.now, sleep=ex.sleep)
    bad = {3, 5}
    assert sorted(j.id for j in srv.failed) == sorted(bad)
    assert "rejected" in jobs[3].error and jobs[3].result is None and jobs[3].offset is None
    assert "non-finite" in jobs[5].error and jobs[5].result is None
    for j in jobs:
        if j.id not in bad:
            assert j.error is None and j.result["steps"] == j.steps
    # job 5 failed inside a quantum that others shared, and later jobs ran
    adv = [e for e in ex.log if e[0] == "advance"]
    assert any(5 in e[2] and len(e[2]) > 1 for e in adv)
    assert not any(5 in e[2] for e in adv[[k for k, e in enumerate(adv) if 5 in e[2]][-1] + 1:])
    assert srv.arena.used == 0 and not srv.busy and not ex.resident
    rep = S.report(jobs, elapsed)
    assert rep["jobs"] == 8 and rep["failed_jobs"] == 2


def test_set_up_and_readout_on_a_worker_thread():
    """Set-ups and readouts that finish later than they were started (on a
    worker thread, as the GPU executor runs them): every job still runs
    exactly its steps, a job is stepped only after its set-up has finished,
    its arena slot is freed only after its result has been read, and a
    rejected set-up and a failed readout each retire their job alone."""

    class Worker(S.ModelExecutor):
        def __init__(self):
            super().__init__(rate=1e9, overhead=1e-4, fail_start={4})
            self.pool = ThreadPoolExecutor(max_workers=1)
            self.lock = threading.Lock()
            self.set_up, self.read = set(), set()

        def start_async(self, job, offset):
            def run():
                time.sleep(0.001)
                with self.lock:
                    r = self.start(job, offset)
                    self.set_up.add(job.id)
                    return r
            return self.pool.submit(run)

        def finish_async(self, job, clock=None):
            def run():
                time.sleep(0.001)
                with self.lock:
                    out = self.finish(job)
                    self.read.add(job.id)
                    if job.id == 6:
                        raise RuntimeError("readout of job 6 failed")
                    return out, None
            return self.pool.submit(run)

        def advance(self, n):
            with self.lock:
                assert self.members <= self.set_up  # never a job still being set up
                return super().advance(n)

    ex = Worker()
    srv = S.Server(ex, 100 << 20, quantum=10)
    jobs = [job(k, (40, 40, 40), 30 + 7 * k) for k in range(8)]
    freed = []
    orig_free = srv.arena.free

    def free(off):
        # every job that held this slot and got past its set-up has been read
        owners = [j.id for j in jobs if j.offset == off and j.id in ex.set_up]
        freed.append((off, [i for i in owners if i not in ex.read]))
        orig_free(off)

    srv.arena.free = free
    S.run_stream(srv, jobs, [0.0003 * k for k in range(8)], clock=ex.now, sleep=ex.sleep)
    ex.pool.shutdown()
    assert "rejected" in jobs[4].error and jobs[4].result is None
    assert "readout of job 6 failed" in jobs[6].error and jobs[6].result is None
    for j in jobs:
        if j.id not in (4, 6):
            assert j.error is None and j.result["steps"] == j.steps
    assert all(not early for _, early in freed)  # no slot freed before its readout
    assert srv.arena.used == 0 and not srv.busy and not ex.resident
