#!/usr/bin/env python3
"""Throughput of the diffuse-solid ternary lattice Boltzmann step on one GPU.

One "step" is one fluid-stage time step of the whole lattice (Sec. II.B of
the paper: stream g and take its moment, chemical potential, forces, stream f
with interpolated bounce-back, velocity, both collisions), run by the fused
gfx950 kernel of libdsm.so through its C ABI.

Headline workload: the D3Q19 micropillar lattice, 256 x 256 x 192 periodic,
an 8-node base slab carrying 16 x 16 square pillars (width 8, pitch 16,
height 32, seeded +-2-node jitter), its diffuse solid relaxed on the GPU by
the solid stage of Sec. II.B (5000 steps from the sharp mask, beta = 1e-3,
Omega = 2e-4), a liquid slab above the pillars (z in [44, 104)), kappa for a
120 degree Young angle (gamma_12 = gamma_23 = 2.5e-3), tau = 1, M = 0.1,
body force -1e-5 along z on the liquid; FP32 populations, with FP16 storage
beside it.  The 128^3 sessile-drop lattice is reported as a second block.
Inputs are resident in HBM when the timed region starts.

Prints ONE JSON line with MLUPS, the roofline of the fused kernel (HBM bytes
of one launch over its event-timed duration), the HBM traffic measured
by rocprofv3 counters when the committed counter summary still matches the
kernel source, streaming-kernel ceilings measured in the same run, the
batched and served forms, and the FP64 CPU oracle timed on this host as a
baseline with the GPU's error against it.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
METRIC = "MLUPS and HBM GB/s (% peak), FP32 vs FP16-store; p50/p99 job latency"
PMC_SUMMARY = {
    "pillars": os.path.join(ROOT, "profiles", "fused_step_d3q19_256x256x192_pillars_pmc.md"),
    "sessile": os.path.join(ROOT, "profiles", "fused_step_d3q19_128cube_pmc.md"),
    "batch": os.path.join(ROOT, "profiles", "batch_step_d2q9_512_lattices_pmc.md"),
}
KERNEL_SOURCES = ["dsm_fused.hip", "dsm_lattice.h", "dsm_internal.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_19941_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_node(Q: int, pop_bytes: int, solid: bool) -> int:
    """Algorithmic HBM bytes the fused kernel moves for one node: every g
    population read once and written once (the Q - 1 moving ones at pop_bytes,
    the rest population in FP64), the same for f at fluid nodes (a solid node
    has no f), and one read of the frozen C1."""
    g = 2 * ((Q - 1) * pop_bytes + 8)
    f = 0 if solid else 2 * Q * pop_bytes
    return g + f + 4


def bytes_per_launch(Q: int, pop_bytes: int, fluid_nodes: int, solid_nodes: int) -> int:
    return fluid_nodes * bytes_per_node(Q, pop_bytes, False) + solid_nodes * bytes_per_node(Q, pop_bytes, True)


def measured_traffic(summary: str, workload: str, tag: str = "", tiling=None):
    """HBM bytes per launch of the fused kernel from a committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the factor measured on
    a plain copy kernel; tag "" for FP32 storage, "_fp16" for FP16), or None
    if absent, taken on another workload, on other kernel source or, when the
    summary records it, with another launch shape than ``tiling``."""
    path = PMC_SUMMARY[summary]
    if not os.path.exists(path):
        return None
    text = open(path).read()

    def field(name):
        m = re.search(rf"^{name}:\s*(\S+)", text, re.M)
        return m.group(1) if m else None

    if field("workload") != workload or field("kernel_source_sha256") != kernel_source_hash():
        return None
    recorded = re.search(rf"^tiling{tag}:\s*(\d+)\s+(\d+)", text, re.M)
    if tiling is not None and recorded and (int(recorded.group(1)), int(recorded.group(2))) != tuple(tiling):
        return None
    try:
        return float(field("hbm_bytes_per_launch" + tag))
    except (TypeError, ValueError):
        return None


def cpu_baseline(w, seconds: float):
    """The FP64 oracle on this host's cores, on the same lattice from the same
    initial state, for about ``seconds`` of CPU work.  Returns the report and
    (total steps, oracle C2 after them) for the accuracy check."""
    from oracle.oracle import Oracle
    from paper_2504_19941_amd import workloads as W

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    o = Oracle(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility, gravity=w.gravity,
               threads=threads)
    o.set_solid_field(f32(W.flat(w.C1)))
    o.set_liquid(f32(W.flat(w.C2)))
    t0 = time.perf_counter()
    o.step(1)
    dt = time.perf_counter() - t0
    more = max(0, int(math.ceil(seconds / max(dt, 1e-6))) - 1)
    t0 = time.perf_counter()
    if more:
        o.step(more)
    dt_more = time.perf_counter() - t0
    steps, total = (more, dt_more) if more else (1, dt)
    C2 = o.fields()["C2"]
    o.close()
    # the same oracle on one core, over one or two steps of the same lattice
    single = 1 if w.nodes > 4_000_000 else 2
    o1 = Oracle(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility, gravity=w.gravity,
                threads=1)
    o1.set_solid_field(f32(W.flat(w.C1)))
    o1.set_liquid(f32(W.flat(w.C2)))
    t0 = time.perf_counter()
    o1.step(single)
    dt1 = time.perf_counter() - t0
    o1.close()
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    report = {
        "value": round(w.nodes * steps / total / 1e6, 4),
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{w.name}: {steps} FP64 oracle steps after 1 untimed, {threads} OpenMP threads, "
                  f"{total:.1f} s; single core: {single} step(s), {dt1:.1f} s",
        "single_core_MLUPS": round(w.nodes * single / dt1 / 1e6, 4),
        "host_cpus": os.cpu_count(),
        "cpu_model": model,
    }
    return report, 1 + more, C2


def f32(a):
    import numpy as np

    return np.asarray(a, dtype=np.float32).astype(np.float64)


def run_storage(dsm, W, w, dev, storage, args, fluid_nodes, solid_nodes, tune_tiling=False):
    """Times the step for one population storage mode: timed region 1 is K
    whole steps bracketed by events (throughput), timed region 2 the same with
    HIP events around every launch (per-launch kernel duration)."""
    import torch

    sim = dsm.Simulation(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                         gravity=w.gravity, reduce_every=0, device=dev, storage=storage)
    if args.tile is not None or args.planes is not None:
        sim.set_tiling(args.tile or 0, args.planes or 16)
    sim.set_solid_field(f32(W.flat(w.C1)))
    sim.set_liquid(f32(W.flat(w.C2)))
    m0 = sim.mass()
    stream = sim.stream
    sim.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1) / max(args.steps, 1)
    fused_ms, links_ms = sim.step_timed(args.steps)
    m1 = sim.mass()
    tiling = sim.tiling()
    tuned = None
    if tune_tiling:
        # the measured tiling tuner on the same lattice, beside the default
        v, planes, tms = sim.tune_tiling(reps=3)
        tuned = {"tiling": [v, planes], "fused_kernel_us": round(tms * 1e3, 2),
                 "default_tiling": list(tiling), "default_fused_kernel_us": round(fused_ms * 1e3, 2)}
    sim.close()
    pop_bytes = 2 if storage == dsm.DSM_STORAGE_FP16 else 4
    alg = bytes_per_launch(19 if w.dim == 3 else 9, pop_bytes, fluid_nodes, solid_nodes)
    return {
        "mlups": w.nodes / (ms * 1e-3) / 1e6,
        "ms": ms,
        "wall": wall,
        "fused_ms": fused_ms,
        "links_ms": links_ms,
        "alg_bytes": alg,
        "achieved": alg / (fused_ms * 1e-3) / 1e9,
        "drift": abs(m1[1] - m0[1]) / abs(m0[1]),
        "tiling": tiling,
        "tuned": tuned,
    }


def run_batch(dsm, W, dev, args):
    """Batched form on many uneven D2Q9 lattices (drops on sinusoidal walls):
    the same lattices stepped (a) one after another by the single-lattice
    launches and (b) together by the tuned persistent batch, replayed
    from a HIP graph.  Both are timed with events over K steps."""
    import numpy as np
    import torch

    ws = W.batch_2d_sinusoid(args.batch_count)
    sims = []
    fluid = solid = 0
    for w in ws:
        s = dsm.Simulation(2, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                           gravity=w.gravity, device=dev)
        s.set_solid_field(f32(W.flat(w.C1)))
        s.set_liquid(f32(W.flat(w.C2)))
        s.step(1)
        ns = int((np.asarray(w.C1, dtype=np.float32) > 0.5).sum())
        solid += ns
        fluid += w.nodes - ns
        sims.append(s)
        if len(sims) % 128 == 0:
            print(f"bench.py: batched form: {len(sims)} lattices set up", file=sys.stderr, flush=True)
    nodes = fluid + solid
    print(f"bench.py: batched form: {len(sims)} lattices, {nodes} nodes set up", file=sys.stderr, flush=True)
    stream = sims[0].stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # (a) one lattice after another
    for s in sims:
        s.step(2)
    torch.cuda.synchronize()
    e0.record(stream)
    for s in sims:
        s.step(args.batch_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / args.batch_steps
    print(f"bench.py: batched form: one lattice at a time {plain_ms:.3f} ms/step", file=sys.stderr, flush=True)
    # (b) batched: the modelled tuner's schedule, then the measured tuner's
    batch = dsm.Batch(sims, device=dev)
    tune_t0 = time.perf_counter()
    cost2, _ = batch.tune()
    tune_s = time.perf_counter() - tune_t0
    batch.step(args.warmup)
    model_sched = batch.schedule(2)
    model_ms = batch.step_timed(args.batch_steps)
    print(f"bench.py: batched form: modelled schedule {model_sched} {model_ms:.4f} ms/step", file=sys.stderr,
          flush=True)
    steps0 = sims[0].steps
    mtune_t0 = time.perf_counter()
    measured_ms, _ = batch.tune(reps=5)
    mtune_s = time.perf_counter() - mtune_t0
    tune_steps = sims[0].steps - steps0
    print(f"bench.py: batched form: measured tuner {batch.schedule(2)} {measured_ms:.4f} ms/step "
          f"({tune_steps} steps, {mtune_s:.2f} s)", file=sys.stderr, flush=True)
    batch.step(args.warmup)
    wall0 = time.perf_counter()
    ms = batch.step_timed(args.batch_steps)
    wall = time.perf_counter() - wall0
    alg = bytes_per_launch(9, 4, fluid, solid)
    out = {
        "workload": f"{len(ws)} D2Q9 lattices {W.BATCH_2D_RECIPE}",
        "nodes": nodes,
        "fluid_node_fraction": round(fluid / nodes, 4),
        "value": round(nodes / (ms * 1e-3) / 1e6, 2),
        "unit": "MLUPS",
        "ms_per_step": round(ms, 5),
        "steps": args.batch_steps,
        "wall_s_timed": round(wall, 4),
        "hbm_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
        "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "algorithmic_bytes": alg,
        "traffic": measured_traffic("batch", "d2q9-512-sinusoid-batch", "",
                                    (batch.schedule(2)["variant"], batch.schedule(2)["planes"])),
        "schedule": batch.schedule(2),
        "tuner": "measured (every candidate timed on the batch itself, 5 steps each)",
        "tune_s": round(mtune_s, 3),
        "tune_steps": tune_steps,
        "items": batch.items(2),
        "modelled_choice": {"schedule": model_sched, "modelled_cost": round(cost2, 1), "tune_s": round(tune_s, 4),
                            "value": round(nodes / (model_ms * 1e-3) / 1e6, 2), "ms_per_step": round(model_ms, 5)},
        "one_lattice_at_a_time": {"value": round(nodes / (plain_ms * 1e-3) / 1e6, 2), "unit": "MLUPS",
                                  "ms_per_step": round(plain_ms, 5)},
        "speedup_vs_one_at_a_time": round(plain_ms / ms, 3),
    }
    batch.close()
    for s in sims:
        s.close()
    return out


def run_serve(dsm, W, dev, args, plain_mlups):
    """Served form: a Poisson stream of 3D jobs of two kinds, FP16 storage on
    a seeded coin, admitted by footprint into one device arena and advanced
    together in quanta by the batched step; latency is arrival to result on
    the host clock (admission set-up, the steps, and the copy of the result
    included).  For a seeded sample of jobs the same work is also timed alone
    (set-up, steps, result copy) to give each job's slowdown in the mix, and
    the smallest job is returned for the oracle replay of the CPU-baseline
    leg."""
    import numpy as np
    import torch

    from paper_2504_19941_amd import serve as S

    pairs = W.serve_jobs(args.serve_jobs, seed=5, steps=(200, 1000))
    coin = np.random.default_rng(7).uniform(size=len(pairs)) < 0.5
    jobs = [S.Job(k, w, n, storage=dsm.DSM_STORAGE_FP16 if coin[k] else dsm.DSM_STORAGE_FP32)
            for k, (w, n) in enumerate(pairs)]
    mean_work = sum(j.nodes * j.steps for j in jobs) / len(jobs)
    rate = args.serve_load * args.serve_capacity_lups / mean_work
    arrivals = S.poisson_arrivals(len(jobs), rate, seed=6)
    cap = int(args.serve_gib * (1 << 30))
    srv = S.make_gpu_server(cap, quantum=args.serve_quantum, device=dev)
    print(f"bench.py: served form: {len(jobs)} jobs, {rate:.2f} arrivals/s, arena {args.serve_gib} GiB",
          file=sys.stderr, flush=True)
    elapsed = S.run_stream(srv, jobs, arrivals)
    rep = S.report(jobs, elapsed)
    peak_gib, rounds = srv.arena.peak / (1 << 30), srv.rounds
    srv.ex.close()
    del srv
    torch.cuda.empty_cache()

    # each sampled job alone: the same set-up, steps and result copy
    sample = sorted(np.random.default_rng(8).choice(len(jobs), size=min(16, len(jobs)), replace=False))
    slow = []
    for k in sample:
        j = jobs[k]
        w = j.workload
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim = dsm.Simulation(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                             gravity=w.gravity, storage=j.storage, rho=w.rho, tau_gas=w.tau_gas or 0.0,
                             device=dev)
        sim.set_solid_field(W.flat(w.C1))
        sim.set_liquid(W.flat(w.C2))
        sim.step(j.steps)
        sim.diagnostics()
        sim.fields(("C2",))
        alone = time.perf_counter() - t0
        sim.close()
        slow.append(j.latency / alone)
    print(f"bench.py: served form: {len(sample)} jobs timed alone", file=sys.stderr, flush=True)

    rep.update({
        "workload": W.SERVE_RECIPE + "; steps 200-1000; FP16 storage on a seeded 50 % coin",
        "fp16_jobs": int(coin.sum()),
        "arrival_rate_per_s": round(rate, 3),
        "offered_load": args.serve_load,
        "arena_GiB": args.serve_gib,
        "quantum_steps": args.serve_quantum,
        "peak_arena_GiB": round(peak_gib, 3),
        "rounds": rounds,
        "unit": "s (latency), MLUPS (aggregate)",
        "aggregate_vs_plain_fp32": round(rep["aggregate_mlups"] / plain_mlups, 3),
        "slowdown_vs_alone": {"jobs": len(sample), "p50": round(float(np.percentile(slow, 50)), 3),
                              "p99": round(float(np.percentile(slow, 99)), 3),
                              "definition": "latency in the mix (arrival to result) over the same job's "
                                            "set-up + steps + result copy run alone"},
    })
    return rep, min(jobs, key=lambda j: j.nodes * j.steps)


def served_job_error(dsm, W, job):
    """The served job replayed alone on the FP64 oracle: max |dC2| of the
    served result."""
    import numpy as np

    from oracle.oracle import Oracle

    w = job.workload
    o = Oracle(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility, gravity=w.gravity,
               rho=w.rho, tau_gas=w.tau_gas, threads=16)
    o.set_solid_field(f32(W.flat(w.C1)))
    o.set_liquid(f32(W.flat(w.C2)))
    o.step(job.steps)
    err = float(np.abs(o.fields()["C2"] - job.result["C2"]).max())
    o.close()
    return {"job": w.name, "steps": job.steps,
            "storage": "fp16" if job.storage == dsm.DSM_STORAGE_FP16 else "fp32", "max_abs_dC2": err}


def error_vs_oracle(dsm, W, w, dev, storage, steps, C2_oracle):
    import numpy as np

    sim = dsm.Simulation(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                         gravity=w.gravity, reduce_every=0, device=dev, storage=storage)
    sim.set_solid_field(f32(W.flat(w.C1)))
    sim.set_liquid(f32(W.flat(w.C2)))
    sim.step(steps)
    err = float(np.abs(sim.fields()["C2"] - C2_oracle).max())
    sim.close()
    return err


def pillar_workload(dsm, W, dev):
    """The micropillar lattice with its diffuse solid from the solid stage on
    the GPU (FP32 storage, from the sharp mask, the stage-1 schedule of the
    workload); returns the workload with C1 set and the liquid slab cut by
    (1 - C1), and the solid stage's duration."""
    import numpy as np
    import torch

    w = W.config_3d_pillars()
    sim = dsm.Simulation(3, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility, gravity=w.gravity,
                         mask=W.flat(w.mask), reduce_every=0, device=dev)
    st = w.solid_stage
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.init_solid(st["n_steps"], st["beta"], st["omega"], 1.0, 1.0 / 6.0, dsm.DSM_SOLID_RESET)
    torch.cuda.synchronize()
    solid_s = time.perf_counter() - t0
    C1 = W.unflat(sim.fields()["C1"], w.shape)
    sim.close()
    torch.cuda.empty_cache()
    w.C1 = C1
    w.C2 = np.asarray(w.C2) * (1.0 - C1)
    print(f"bench.py: {w.name}: solid stage {st['n_steps']} steps in {solid_s:.2f} s", file=sys.stderr, flush=True)
    return w, solid_s


def stream_reference(dev):
    """Achievable bandwidth in the same run: torch's device copy and fill of
    1 GiB, and the streaming kernels of libdsm_probe.so (16 bytes per lane,
    grid-stride; copy with plain and non-temporal stores, read only, write
    only) over a sweep of grid sizes, best of five each."""
    import ctypes

    import torch

    from paper_2504_19941_amd import build as B

    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev)

    def best_ms(fn):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(5):
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            fn()
            s1.record(stream)
            torch.cuda.synchronize()
            t.append(s0.elapsed_time(s1))
        return min(t)

    tc, tf = best_ms(lambda: b.copy_(a)), best_ms(lambda: b.fill_(2.0))
    out = {"torch": {"kind": "copy_ and fill_ of 1 GiB, best of 5",
                     "copy_GBps": round(2 * (1 << 30) / (tc * 1e-3) / 1e9, 1),
                     "fill_GBps": round((1 << 30) / (tf * 1e-3) / 1e9, 1)}}
    if os.path.exists(B.PROBE_LIB):
        lib = ctypes.CDLL(B.PROBE_LIB)
        lib.dsm_probe_stream.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_int, ctypes.c_void_p]
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        nbytes = 1 << 30
        probe = {}
        for kind, name, moved in ((0, "copy", 2), (1, "copy_nt", 2), (4, "copy4", 2), (2, "read", 1),
                                  (3, "write", 1)):
            best = None
            for per_cu in (4, 8, 16, 32):
                blocks = cus * per_cu

                def go():
                    rc = lib.dsm_probe_stream(kind, a.data_ptr(), b.data_ptr(), nbytes, blocks,
                                              ctypes.c_void_p(stream.cuda_stream))
                    if rc != 0:
                        raise RuntimeError(f"dsm_probe_stream failed ({rc})")

                ms = best_ms(go)
                gbps = moved * nbytes / (ms * 1e-3) / 1e9
                if best is None or gbps > best[0]:
                    best = (gbps, per_cu)
            probe[name + "_GBps"] = round(best[0], 1)
            probe[name + "_blocks_per_cu"] = best[1]
        probe["kind"] = ("libdsm_probe.so: 16 B per lane (copy4: 4 B per lane), grid-stride, 1 GiB, best of 5 "
                         "over 4-32 blocks per CU")
        out["probe"] = probe
    del a, b
    torch.cuda.empty_cache()
    copies = [out["torch"]["copy_GBps"]] + ([out["probe"]["copy_GBps"], out["probe"]["copy_nt_GBps"]]
                                              if "probe" in out else [])
    out["best_copy_GBps"] = max(copies)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tile", type=int, default=None, help="fused-kernel tile variant")
    ap.add_argument("--planes", type=int, default=None, help="planes marched per workgroup")
    ap.add_argument("--no-sessile", action="store_true", help="skip the 128^3 sessile-drop block")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--batch-count", type=int, default=512, help="lattices in the batched-form measurement")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--serve-gib", type=float, default=16.0, help="device arena of the served form")
    ap.add_argument("--serve-quantum", type=int, default=50, help="steps per round of the served form")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="offered load: arrival rate x mean job work / --serve-capacity-lups")
    ap.add_argument("--serve-capacity-lups", type=float, default=12e9)
    ap.add_argument("--no-stream-reference", action="store_true", help="skip the copy/read/write references")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, run 3 plain device copies of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the benchmark runs the step on one GPU "
              "(a lattice would shard by slabs with one halo exchange per step; that path is not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2504_19941_amd import dsm
    from paper_2504_19941_amd import workloads as W

    dsm.load()  # raises if libdsm.so is missing: there is no fallback
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def storage_block(r, alg_nodes):
        return {"value": round(r["mlups"], 2), "unit": "MLUPS", "ms_per_step": round(r["ms"], 5),
                "fused_kernel_us": round(r["fused_ms"] * 1e3, 2), "link_kernel_us": round(r["links_ms"] * 1e3, 2),
                "hbm_GBps": round(r["achieved"], 1), "hbm_frac": round(r["achieved"] / HBM_PEAK_GBPS, 4),
                "algorithmic_bytes": r["alg_bytes"], "tiling": list(r["tiling"]),
                "liquid_mass_drift_rel": r["drift"], **({"tiling_tuner": r["tuned"]} if r["tuned"] else {})}

    # headline: the micropillar lattice, FP32 and FP16 storage
    w, solid_s = pillar_workload(dsm, W, dev)
    solid_nodes = int((np.asarray(w.C1, dtype=np.float32) > 0.5).sum())
    fluid_nodes = w.nodes - solid_nodes
    r32 = run_storage(dsm, W, w, dev, dsm.DSM_STORAGE_FP32, args, fluid_nodes, solid_nodes, tune_tiling=True)
    r16 = run_storage(dsm, W, w, dev, dsm.DSM_STORAGE_FP16, args, fluid_nodes, solid_nodes, tune_tiling=True)
    print(f"bench.py: {w.name}: fp32 {r32['mlups']:.0f} MLUPS, fp16 {r16['mlups']:.0f} MLUPS",
          file=sys.stderr, flush=True)

    # second block: the 128^3 sessile drop
    sessile = None
    if not args.no_sessile:
        ws = W.config_3d_sessile(90.0, n=128)
        s_solid = int((np.asarray(ws.C1, dtype=np.float32) > 0.5).sum())
        s32 = run_storage(dsm, W, ws, dev, dsm.DSM_STORAGE_FP32, args, ws.nodes - s_solid, s_solid)
        s16 = run_storage(dsm, W, ws, dev, dsm.DSM_STORAGE_FP16, args, ws.nodes - s_solid, s_solid)
        sessile = storage_block(s32, ws.nodes)
        sessile.update({"workload": ws.name, "shape": list(ws.shape),
                        "fluid_node_fraction": round((ws.nodes - s_solid) / ws.nodes, 4),
                        "traffic": measured_traffic("sessile", ws.name, "", s32["tiling"])})
        sessile["fp16_store"] = storage_block(s16, ws.nodes)
        sessile["fp16_store"]["traffic"] = measured_traffic("sessile", ws.name, "_fp16", s16["tiling"])
        sessile["fp16_store"]["speedup_vs_fp32"] = round(s16["mlups"] / s32["mlups"], 3)

    stream_ref = None if args.no_stream_reference else stream_reference(dev)

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    N = w.nodes
    achieved = r32["achieved"]
    out = {
        "metric": METRIC,
        "value": round(r32["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "lattice": "D3Q19",
            "shape": list(w.shape),
            "solid": "16x16 square pillars (width 8, pitch 16, height 32, seeded +-2 jitter) on an 8-node "
                     "base; C1 from the solid stage on the GPU (5000 steps, beta 1e-3, Omega 2e-4)",
            "liquid": "slab z in [44, 104) above the pillars, body force -1e-5 along z",
            "storage": "fp32 (fp16 in fp16_store)",
            "fluid_node_fraction": round(fluid_nodes / N, 4),
            "theta_deg": 120.0,
            "tau": w.tau,
            "mobility": w.mobility,
            "kappa": [round(k, 8) for k in w.kappa],
            "tiling": list(r32["tiling"]),
        },
        "solid_stage_s": round(solid_s, 3),
        "hbm_GBps": round(achieved, 1),
        "hbm_frac": round(achieved / HBM_PEAK_GBPS, 4),
        "fused_kernel_us": round(r32["fused_ms"] * 1e3, 2),
        "link_kernel_us": round(r32["links_ms"] * 1e3, 2),
        "liquid_mass_drift_rel": r32["drift"],
        "wall_s_timed": round(r32["wall"], 4),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic("pillars", w.name, "", r32["tiling"]),
            "algorithmic_bytes": r32["alg_bytes"],
            # the same count with every node charged as a fluid node (solid
            # nodes' f traffic not skipped)
            "without_solid_skip": {
                "algorithmic_bytes": N * bytes_per_node(19, 4, False),
                "achieved": round(N * bytes_per_node(19, 4, False) / (r32["fused_ms"] * 1e-3) / 1e9, 1),
                "frac": round(N * bytes_per_node(19, 4, False) / (r32["fused_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            },
            "kernel": "k_step_fused<3,...> (one launch per step), 256x256x192 pillars, FP32",
            "stream_reference": stream_ref,
            "frac_of_best_copy": round(achieved / stream_ref["best_copy_GBps"], 4) if stream_ref else None,
            "tiling_tuner": r32["tuned"],
        },
    }
    out["fp16_store"] = storage_block(r16, N)
    out["fp16_store"]["traffic"] = measured_traffic("pillars", w.name, "_fp16", r16["tiling"])
    out["fp16_store"]["speedup_vs_fp32"] = round(r16["mlups"] / r32["mlups"], 3)
    if sessile is not None:
        out["d3q19_128cube"] = sessile
    if not args.no_batch:
        out["batched_2d"] = run_batch(dsm, W, dev, args)
    small_job = None
    if not args.no_serve:
        out["served_3d"], small_job = run_serve(dsm, W, dev, args, r32["mlups"])
    if not args.no_cpu_baseline:
        report, steps, C2o = cpu_baseline(w, args.cpu_seconds)
        out["cpu_baseline"] = report
        out["error_vs_oracle"] = {
            "workload": w.name,
            "steps": steps,
            "fp32_max_abs_dC2": error_vs_oracle(dsm, W, w, dev, dsm.DSM_STORAGE_FP32, steps, C2o),
            "fp16_max_abs_dC2": error_vs_oracle(dsm, W, w, dev, dsm.DSM_STORAGE_FP16, steps, C2o),
        }
        if small_job is not None:
            out["served_3d"]["error_vs_oracle"] = served_job_error(dsm, W, small_job)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
