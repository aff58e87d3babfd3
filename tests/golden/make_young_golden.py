"""Writes tests/golden/young_d2q9_128x64_theta<T>.json: the FP64 oracle's contact
angle history for the D2Q9 128 x 64 sessile drop (8-node wall, R = 25,
tau = 1, M = 0.1, gamma = 2.5e-3) at 60, 90 and 120 degrees.

Calls only the oracle (plus the seeded input generator and the angle fit).
Usage:  python tests/golden/make_young_golden.py [steps] [theta ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.oracle import Oracle  # noqa: E402
from paper_2504_19941_amd import analysis as A  # noqa: E402
from paper_2504_19941_amd import workloads as W  # noqa: E402

EVERY = 2000


def run(theta, steps, threads=2):
    w = W.config_2d_contact_angle(theta)
    o = Oracle(2, w.shape, w.kappa, mobility=w.mobility, tau=w.tau, threads=threads)
    o.set_solid_field(W.flat(w.C1))
    o.set_liquid(W.flat(w.C2))
    m0 = o.mass()
    hist = []
    t0 = time.time()
    for k in range(steps // EVERY):
        o.step(EVERY)
        fl = o.fields()
        th = A.contact_angle(W.unflat(fl["C1"], w.shape), W.unflat(fl["C2"], w.shape), 1, w.wall_level)
        F, E = o.free_energy()
        hist.append({"step": (k + 1) * EVERY, "theta": th, "F": F, "Ekin": E,
                     "umax": float(abs(fl["u"]).max())})
        print(theta, (k + 1) * EVERY, round(th, 3), round(time.time() - t0), flush=True)
    m1 = o.mass()
    return {"theta_target": theta, "kappa": list(w.kappa), "mass0": list(m0), "mass1": list(m1),
            "history": hist}


if __name__ == "__main__":
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 200000
    thetas = [float(t) for t in sys.argv[2:]] or [60.0, 90.0, 120.0]
    for th in thetas:
        data = run(th, steps)
        data["about"] = ("FP64 oracle, D2Q9 128x64 periodic, wall rows y<=7 (analytic tanh, face "
                          "y=7.5), semicircular drop R=25 at x=64, tau=1, M=0.1, gamma=2.5e-3; "
                          "written by tests/golden/make_young_golden.py")
        json.dump(data, open(os.path.join(HERE, f"young_d2q9_128x64_theta{th:g}.json"), "w"), indent=1)
