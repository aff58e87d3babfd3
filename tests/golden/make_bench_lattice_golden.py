"""Writes tests/golden/sessile3d_d3q19_128cube_R30_theta60_1000steps.json:
the FP64 oracle's state after 1000 steps of the full-size D3Q19 sessile-drop
lattice (128^3, 6-node slab with an analytic tanh edge, hemispherical drop
R = 30, tau = 1, M = 0.1, gamma = 2.5e-3, target 60 degrees so that the drop
spreads), sampled where the oracle's values can be stored: C2 and u at 1024
seeded random nodes and on the vertical x-z plane through the drop centre
(z < 40), plus the amounts, free energy and kinetic energy.  Inputs are
rounded to FP32 first, as every GPU comparison does.

Calls only the oracle (plus the seeded input generator).
Usage:  python tests/golden/make_bench_lattice_golden.py [threads]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle.oracle import Oracle  # noqa: E402
from paper_2504_19941_amd import workloads as W  # noqa: E402

STEPS, THETA, N = 1000, 60.0, 128
NAME = "sessile3d_d3q19_128cube_R30_theta60_1000steps.json"


def sample_nodes():
    """Flat node indices: 1024 seeded random nodes, then the plane y = 64,
    z < 40 in x-fastest order."""
    rng = np.random.default_rng(1000)
    rnd = rng.choice(N ** 3, size=1024, replace=False)
    x, z = np.meshgrid(np.arange(N), np.arange(40), indexing="xy")
    plane = (x + N * (N // 2 + N * z)).reshape(-1)
    return np.concatenate([np.sort(rnd), plane]).astype(np.int64)


def main(threads):
    w = W.config_3d_sessile(THETA, n=N)
    o = Oracle(3, w.shape, w.kappa, mobility=w.mobility, tau=w.tau, threads=threads)
    o.set_solid_field(np.asarray(W.flat(w.C1), np.float32).astype(np.float64))
    o.set_liquid(np.asarray(W.flat(w.C2), np.float32).astype(np.float64))
    m0 = o.mass()
    t0 = time.time()
    for k in range(STEPS // 100):
        o.step(100)
        print(f"step {(k + 1) * 100} ({time.time() - t0:.0f} s)", flush=True)
    fl = o.fields()
    F, E = o.free_energy()
    idx = sample_nodes()
    def g10(a):  # ten significant digits: far below the 1e-5 comparison bar
        return [float(f"{v:.10g}") for v in a]

    data = {"steps": STEPS, "theta_target": THETA, "kappa": list(w.kappa), "shape": [N, N, N],
            "nodes": idx.tolist(), "C2": g10(fl["C2"][idx]),
            "u": [g10(fl["u"][d][idx]) for d in range(3)],
            "mass0": list(m0), "mass": list(o.mass()), "F": F, "Ekin": E,
            "about": ("FP64 oracle, D3Q19 128^3 periodic, slab z<=5 (analytic tanh, face z=5.5), "
                      "hemispherical drop R=30 at (64, 64, 5.5), tau=1, M=0.1, gamma=2.5e-3, theta 60, "
                      "inputs rounded to FP32, 1000 steps; written by tests/golden/make_bench_lattice_golden.py")}
    out_dir = os.environ.get("GOLDEN_OUT", HERE)
    json.dump(data, open(os.path.join(out_dir, NAME), "w"))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
