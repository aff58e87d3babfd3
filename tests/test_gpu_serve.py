"""Served form on the GPU: jobs of both kinds (capillary ducts with the
paper's liquid/gas viscosity contrast, particles at an interface; FP32 and
FP16 storage) submitted while others run, admitted by
footprint into one device arena, advanced together by the batched step, give
exactly the result each gives alone; and served jobs of each kind and
storage match the FP64 oracle run of the same job."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2504_19941_amd import dsm
from paper_2504_19941_amd import serve as S
from paper_2504_19941_amd import workloads as W

from .conftest import f32

pytestmark = pytest.mark.gpu


def alone(job):
    w = job.workload
    sim = dsm.Simulation(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                         gravity=w.gravity, storage=job.storage, rho=w.rho, tau_gas=w.tau_gas or 0.0)
    sim.set_solid_field(f32(W.flat(w.C1)))
    sim.set_liquid(f32(W.flat(w.C2)))
    sim.step(job.steps)
    out = {"C2": sim.fields()["C2"], "mass": sim.mass(), "steps": sim.steps}
    sim.close()
    return out


def make_jobs(count, seed):
    pairs = W.serve_jobs(count, seed=seed, steps=(15, 70), small=True)
    return [S.Job(k, w, n, storage=dsm.DSM_STORAGE_FP16 if k % 3 == 2 else dsm.DSM_STORAGE_FP32)
            for k, (w, n) in enumerate(pairs)]


def check_alone(jobs):
    for j in jobs:
        ref = alone(j)
        assert j.result["steps"] == j.steps == ref["steps"]
        same = np.array_equal(j.result["C2"], ref["C2"])
        err = float(np.abs(j.result["C2"] - ref["C2"]).max())
        print(f"  job {j.id} {j.workload.name} steps {j.steps} storage {j.storage}: max |dC2| {err:.1e}",
              flush=True)
        assert same, f"job {j.id} differs from its run alone"
        assert np.array_equal(j.result["mass"], ref["mass"])


def test_jobs_joining_mid_run_match_their_runs_alone(gpu):
    jobs = make_jobs(6, seed=21)
    srv = S.make_gpu_server(256 << 20, quantum=7)
    srv.submit(jobs[0], 0.0)
    srv.step(0.0)
    srv.submit(jobs[1], 0.1)
    srv.step(0.1)
    srv.step(0.2)
    for j in jobs[2:]:
        srv.submit(j, 0.3)
    rounds = 0
    while srv.busy:
        srv.step(1.0)
        rounds += 1
        assert rounds < 1000
    assert len(srv.done) == len(jobs)
    check_alone(jobs)


def test_admission_by_footprint_queues_and_completes(gpu):
    """An arena that holds about two of the jobs at once: the rest wait in
    order, and every job still ends exactly as alone."""
    jobs = make_jobs(5, seed=33)
    probe = S.GpuExecutor(1 << 20)
    sizes = [probe.job_bytes(j) for j in jobs]
    del probe
    cap = (16 << 20) + 2 * max(sizes) + (1 << 20)
    srv = S.make_gpu_server(cap, quantum=9)
    for j in jobs:
        srv.submit(j, 0.0)
    peak_jobs = 0
    while srv.busy:
        srv.step(float(srv.rounds))  # the round number serves as the clock
        peak_jobs = max(peak_jobs, len(srv.running))
        assert srv.arena.used <= srv.arena.capacity
    print(f"  footprints {sizes}, arena {srv.arena.capacity}, at most {peak_jobs} resident", flush=True)
    assert 1 <= peak_jobs < len(jobs)
    adm = [j.admitted for j in jobs]
    assert adm == sorted(adm)
    check_alone(jobs)


def test_served_jobs_match_the_oracle(gpu):
    """A mix of eight jobs served together (300-600 steps each, quantum 50):
    a capillary duct with the paper's capillary-filling viscosities
    (tau_3 = 0.52 against tau_2 = 1) and a particle at an interface in FP32,
    within 1e-5 of the oracle's C2 (and u within 1e-6); a duct and a particle
    with FP16 storage within 2e-3."""
    pairs = W.serve_jobs(8, seed=41, steps=(300, 600), small=True)
    storage = {0: dsm.DSM_STORAGE_FP32, 2: dsm.DSM_STORAGE_FP32, 3: dsm.DSM_STORAGE_FP16,
               5: dsm.DSM_STORAGE_FP16}
    jobs = [S.Job(k, w, n, storage=storage.get(k, dsm.DSM_STORAGE_FP32)) for k, (w, n) in enumerate(pairs)]
    srv = S.make_gpu_server(512 << 20, quantum=50)
    for j in jobs:
        srv.submit(j, 0.0)
    rounds = 0
    while srv.busy:
        srv.step(float(rounds))
        rounds += 1
        assert rounds < 1000
    checked = set()
    for k, st in storage.items():
        j = jobs[k]
        w = j.workload
        kind = "duct" if "channel" in w.name else "particle"
        checked.add((kind, st))
        orc = Oracle(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                     gravity=w.gravity, rho=w.rho, tau_gas=w.tau_gas, threads=16)
        orc.set_solid_field(f32(W.flat(w.C1)))
        orc.set_liquid(f32(W.flat(w.C2)))
        orc.step(j.steps)
        fo = orc.fields()
        orc.close()
        err = float(np.abs(j.result["C2"] - fo["C2"]).max())
        bar = 1e-5 if st == dsm.DSM_STORAGE_FP32 else 2e-3
        print(f"  job {k} {w.name} ({kind}, tau_gas {w.tau_gas}) storage {st}, {j.steps} steps: "
              f"max |dC2| vs oracle {err:.2e} (bar {bar:g})", flush=True)
        assert err < bar
    assert checked == {("duct", 0), ("particle", 0), ("duct", 1), ("particle", 1)}


def test_a_job_that_goes_non_finite_is_retired_alone(gpu):
    """One job of a served mix is driven non-finite (a body force of 50 on
    its liquid); the batch step reports it, the job is retired with
    DSM_EUNSTABLE and its slot freed, and every other job, including those
    that shared its quanta, ends exactly as it does alone."""
    import dataclasses

    jobs = make_jobs(5, seed=57)
    w = jobs[1].workload
    bad = S.Job(99, dataclasses.replace(w, gravity=(50.0,) + tuple(w.gravity[1:])), 400,
                storage=jobs[1].storage)
    srv = S.make_gpu_server(512 << 20, quantum=10)
    srv.submit(jobs[0], 0.0)
    srv.submit(bad, 0.0)
    for j in jobs[1:]:
        srv.submit(j, 0.0)
    rounds = 0
    while srv.busy:
        srv.step(float(rounds))
        rounds += 1
        assert rounds < 1000
    print(f"  failed: {[(j.id, j.error) for j in srv.failed]}", flush=True)
    assert [j.id for j in srv.failed] == [99]
    assert "DSM_EUNSTABLE" in bad.error and bad.result is None and bad.done_steps < bad.steps
    assert srv.arena.used == 0
    assert len(srv.done) == len(jobs)
    check_alone(jobs)
