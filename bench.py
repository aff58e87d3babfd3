#!/usr/bin/env python3
"""Throughput of the diffuse-solid ternary lattice Boltzmann step on one GPU.

One "step" is one fluid-stage time step of the whole lattice (Sec. II.B of
the paper: stream g and take its moment, chemical potential, forces, stream f
with interpolated bounce-back, velocity, both collisions), run by the fused
gfx950 kernel of libdsm.so through its C ABI.

Default workload: D3Q19 128^3 periodic box, 6-node diffuse solid slab
(analytic tanh edge, alpha = 1), hemispherical liquid drop of radius 30 on
it, kappa for a 90 degree Young angle (gamma_12 = gamma_23 = 2.5e-3),
tau = 1, M = 0.1, FP32 populations.  Inputs are resident in HBM when the timed
region starts.

Prints ONE JSON line with MLUPS, the roofline of the fused kernel (HBM bytes
of one launch over its event-timed duration), the HBM traffic measured
by rocprofv3 counters when the committed counter summary still matches the
kernel source, and the FP64 CPU oracle timed on this host as a baseline.

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
PMC_SUMMARY = os.path.join(ROOT, "profiles", "fused_step_d3q19_128cube_pmc.md")
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


def measured_traffic(workload: str, nodes: int, tag: str = ""):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the factor measured on
    a plain copy kernel; tag "" for FP32 storage, "_fp16" for FP16), or None
    if absent or taken on other kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()

    def field(name):
        m = re.search(rf"^{name}:\s*(\S+)", text, re.M)
        return m.group(1) if m else None

    if field("workload") != workload or field("kernel_source_sha256") != kernel_source_hash():
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
    o = Oracle(w.dim, w.shape, w.kappa, tau=w.tau, mobility=w.mobility, threads=threads)
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
    # the same oracle on one core, over two steps of the same lattice
    o1 = Oracle(w.dim, w.shape, w.kappa, tau=w.tau, mobility=w.mobility, threads=1)
    o1.set_solid_field(f32(W.flat(w.C1)))
    o1.set_liquid(f32(W.flat(w.C2)))
    t0 = time.perf_counter()
    o1.step(2)
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
                  f"{total:.1f} s; single core: 2 steps, {dt1:.1f} s",
        "single_core_MLUPS": round(w.nodes * 2 / dt1 / 1e6, 4),
        "host_cpus": os.cpu_count(),
        "cpu_model": model,
    }
    return report, 1 + more, C2


def f32(a):
    import numpy as np

    return np.asarray(a, dtype=np.float32).astype(np.float64)


def run_storage(dsm, W, w, dev, storage, args, fluid_nodes, solid_nodes):
    """Times the step for one population storage mode: timed region 1 is K
    whole steps bracketed by events (throughput), timed region 2 the same with
    HIP events around every launch (per-launch kernel duration)."""
    import torch

    sim = dsm.Simulation(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                         reduce_every=0, device=dev, storage=storage)
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
    # (b) batched
    batch = dsm.Batch(sims, device=dev)
    tune_t0 = time.perf_counter()
    cost2, _ = batch.tune()
    tune_s = time.perf_counter() - tune_t0
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
        "schedule": batch.schedule(2),
        "items": batch.items(2),
        "modelled_cost": round(cost2, 1),
        "tune_s": round(tune_s, 3),
        "one_lattice_at_a_time": {"value": round(nodes / (plain_ms * 1e-3) / 1e6, 2), "unit": "MLUPS",
                                  "ms_per_step": round(plain_ms, 5)},
        "speedup_vs_one_at_a_time": round(plain_ms / ms, 3),
    }
    batch.close()
    for s in sims:
        s.close()
    return out


def run_serve(dsm, W, dev, args, plain_mlups):
    """Served form: a Poisson stream of 3D jobs of two kinds admitted by
    footprint into one device arena and advanced together in quanta by the
    batched step; latency is arrival to result on the host clock (admission
    set-up, the steps, and the copy of the result included)."""
    from paper_2504_19941_amd import serve as S

    pairs = W.serve_jobs(args.serve_jobs, seed=5, steps=(200, 1000))
    jobs = [S.Job(k, w, n, storage=dsm.DSM_STORAGE_FP16 if k % 4 == 3 else dsm.DSM_STORAGE_FP32)
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
    rep.update({
        "workload": W.SERVE_RECIPE + f"; steps 200-1000; every 4th job FP16 storage",
        "arrival_rate_per_s": round(rate, 3),
        "offered_load": args.serve_load,
        "arena_GiB": args.serve_gib,
        "quantum_steps": args.serve_quantum,
        "peak_arena_GiB": round(srv.arena.peak / (1 << 30), 3),
        "rounds": srv.rounds,
        "unit": "s (latency), MLUPS (aggregate)",
        "aggregate_vs_plain_fp32_128cube": round(rep["aggregate_mlups"] / plain_mlups, 3),
    })
    return rep


def error_vs_oracle(dsm, W, w, dev, storage, steps, C2_oracle):
    import numpy as np

    sim = dsm.Simulation(w.dim, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility,
                         reduce_every=0, device=dev, storage=storage)
    sim.set_solid_field(f32(W.flat(w.C1)))
    sim.set_liquid(f32(W.flat(w.C2)))
    sim.step(steps)
    err = float(np.abs(sim.fields()["C2"] - C2_oracle).max())
    sim.close()
    return err


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--theta", type=float, default=90.0)
    ap.add_argument("--tile", type=int, default=None, help="fused-kernel tile variant")
    ap.add_argument("--planes", type=int, default=None, help="planes marched per workgroup")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--batch-count", type=int, default=512, help="lattices in the batched-form measurement")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--serve-jobs", type=int, default=48)
    ap.add_argument("--serve-gib", type=float, default=16.0, help="device arena of the served form")
    ap.add_argument("--serve-quantum", type=int, default=50, help="steps per round of the served form")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="offered load: arrival rate x mean job work / --serve-capacity-lups")
    ap.add_argument("--serve-capacity-lups", type=float, default=12e9)
    ap.add_argument("--no-stream-reference", action="store_true", help="skip the torch copy/fill reference")
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

    w = W.config_3d_sessile(args.theta, n=128)
    Q = 19
    solid_nodes = int((np.asarray(w.C1, dtype=np.float32) > 0.5).sum())
    fluid_nodes = w.nodes - solid_nodes
    r32 = run_storage(dsm, W, w, dev, dsm.DSM_STORAGE_FP32, args, fluid_nodes, solid_nodes)
    r16 = run_storage(dsm, W, w, dev, dsm.DSM_STORAGE_FP16, args, fluid_nodes, solid_nodes)

    # achievable-bandwidth reference in the same run: torch's device copy and
    # fill of 1 GiB (read + write, write only), best of five
    stream_ref = None
    if not args.no_stream_reference:
        n = (1 << 30) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)

        def best_ms(fn):
            fn()
            torch.cuda.synchronize()
            t = []
            for _ in range(5):
                s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s0.record()
                fn()
                s1.record()
                torch.cuda.synchronize()
                t.append(s0.elapsed_time(s1))
            return min(t)

        tc, tf = best_ms(lambda: b.copy_(a)), best_ms(lambda: b.fill_(2.0))
        stream_ref = {"kind": "torch copy_ and fill_ of 1 GiB, best of 5",
                      "copy_GBps": round(2 * (1 << 30) / (tc * 1e-3) / 1e9, 1),
                      "fill_GBps": round((1 << 30) / (tf * 1e-3) / 1e9, 1)}
        del a, b
        torch.cuda.empty_cache()

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    N = w.nodes
    ms = r32["ms"]
    mlups = r32["mlups"]
    alg_bytes = r32["alg_bytes"]
    achieved = r32["achieved"]
    fused_ms, links_ms, drift, wall = r32["fused_ms"], r32["links_ms"], r32["drift"], r32["wall"]
    traffic = measured_traffic(w.name, N)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "lattice": "D3Q19",
            "shape": list(w.shape),
            "storage": "fp32 (fp16 in fp16_store)",
            "fluid_node_fraction": round(fluid_nodes / N, 4),
            "tau": w.tau,
            "mobility": w.mobility,
            "kappa": [round(k, 8) for k in w.kappa],
        },
        "hbm_GBps": round(achieved, 1),
        "hbm_frac": round(achieved / HBM_PEAK_GBPS, 4),
        "fused_kernel_us": round(fused_ms * 1e3, 2),
        "link_kernel_us": round(links_ms * 1e3, 2),
        "liquid_mass_drift_rel": drift,
        "wall_s_timed": round(wall, 4),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "algorithmic_bytes": alg_bytes,
            "kernel": "k_step_fused<3,...> (one launch per step)",
            "stream_reference": stream_ref,
            "frac_of_stream_copy": round(achieved / stream_ref["copy_GBps"], 4) if stream_ref else None,
        },
    }
    out["fp16_store"] = {
        "value": round(r16["mlups"], 2),
        "unit": "MLUPS",
        "ms_per_step": round(r16["ms"], 5),
        "fused_kernel_us": round(r16["fused_ms"] * 1e3, 2),
        "link_kernel_us": round(r16["links_ms"] * 1e3, 2),
        "hbm_GBps": round(r16["achieved"], 1),
        "hbm_frac": round(r16["achieved"] / HBM_PEAK_GBPS, 4),
        "algorithmic_bytes": r16["alg_bytes"],
        "speedup_vs_fp32": round(r16["mlups"] / r32["mlups"], 3),
        "traffic": measured_traffic(w.name, N, "_fp16"),
        "liquid_mass_drift_rel": r16["drift"],
    }
    if not args.no_batch:
        out["batched_2d"] = run_batch(dsm, W, dev, args)
    if not args.no_serve:
        out["served_3d"] = run_serve(dsm, W, dev, args, mlups)
    if not args.no_cpu_baseline:
        report, steps, C2o = cpu_baseline(w, args.cpu_seconds)
        out["cpu_baseline"] = report
        out["error_vs_oracle"] = {
            "steps": steps,
            "fp32_max_abs_dC2": error_vs_oracle(dsm, W, w, dev, dsm.DSM_STORAGE_FP32, steps, C2o),
            "fp16_max_abs_dC2": error_vs_oracle(dsm, W, w, dev, dsm.DSM_STORAGE_FP16, steps, C2o),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
