"""Writes tests/golden/sessile3d_d3q19_64cube_R15_theta<T>.json: the FP64
oracle's history of a D3Q19 sessile drop, the 64^3 / R = 15 reduction of the
128^3 / R = 30 contact-angle workload (6-node slab with an analytic tanh
edge, face at z = 5.5, hemispherical drop centred on the face, tau = 1,
M = 0.1, gamma = 2.5e-3), at target angles 60, 90 and 120 degrees.

Every EVERY steps it records the sphere-fit contact angle, the free and
kinetic energies, the largest speed and the three amounts; at the end it
stores C2 on two lines through the drop (the vertical axis and the x line
two nodes above the wall face through the centre).  Inputs are rounded to
FP32 first, as every GPU comparison does.

Calls only the oracle (plus the seeded input generator and the angle fit).
Usage:  python tests/golden/make_sessile3d_golden.py [steps] [threads] [theta ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle.oracle import Oracle  # noqa: E402
from paper_2504_19941_amd import analysis as A  # noqa: E402
from paper_2504_19941_amd import workloads as W  # noqa: E402

EVERY = 2500
N, R = 64, 15.0


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def workload(theta):
    return W.config_3d_sessile(theta, n=N, radius=R)


def lines(C2, shape, face):
    c = W.unflat(C2, shape)
    zc = int(round(face + 2.0))
    return {"axis_z": c[N // 2, N // 2, :].tolist(), "line_x_z%d" % zc: c[:, N // 2, zc].tolist()}


def run(theta, steps, threads, out=None):
    """Runs the oracle; when ``out`` is given, rewrites that file after every
    record, so that an interrupted run still leaves a valid shorter history."""
    w = workload(theta)
    o = Oracle(3, w.shape, w.kappa, mobility=w.mobility, tau=w.tau, threads=threads)
    o.set_solid_field(f32(W.flat(w.C1)))
    o.set_liquid(f32(W.flat(w.C2)))
    m0 = o.mass()
    hist = []
    t0 = time.time()
    for k in range(steps // EVERY):
        for part in range(EVERY // 500):
            o.step(500)
            print(f"theta {theta:g}: step {k * EVERY + (part + 1) * 500} ({time.time() - t0:.0f} s)", flush=True)
        fl = o.fields()
        th = A.contact_angle(W.unflat(fl["C1"], w.shape), W.unflat(fl["C2"], w.shape), 2, w.wall_level)
        F, E = o.free_energy()
        u = fl["u"]
        hist.append({"step": (k + 1) * EVERY, "theta": th, "F": F, "Ekin": E,
                     "umax": float(np.sqrt((u ** 2).sum(axis=0)).max()), "mass": list(o.mass())})
        print(f"theta {theta:g}: step {(k + 1) * EVERY} angle {th:.3f} ({time.time() - t0:.0f} s)", flush=True)
        data = {"theta_target": theta, "kappa": list(w.kappa), "shape": list(w.shape), "radius": R,
                "wall_level": w.wall_level, "mass0": list(m0), "history": hist,
                "final_lines": lines(fl["C2"], w.shape, w.wall_level),
                "about": ("FP64 oracle, D3Q19 64^3 periodic, slab z<=5 (analytic tanh, face z=5.5), "
                          "hemispherical drop R=15 at (32, 32, 5.5), tau=1, M=0.1, gamma=2.5e-3, inputs "
                          "rounded to FP32; written by tests/golden/make_sessile3d_golden.py")}
        if out:
            tmp = out + ".tmp"
            json.dump(data, open(tmp, "w"), indent=1)
            os.replace(tmp, out)
    return data


def path(theta):
    return os.path.join(HERE, f"sessile3d_d3q19_64cube_R15_theta{theta:g}.json")


if __name__ == "__main__":
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 20000
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 4
    thetas = [float(t) for t in sys.argv[3:]] or [60.0, 90.0, 120.0]
    out_dir = os.environ.get("GOLDEN_OUT", HERE)
    for th in thetas:
        run(th, steps, threads, out=os.path.join(out_dir, os.path.basename(path(th))))
