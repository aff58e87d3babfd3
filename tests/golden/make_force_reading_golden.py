"""Writes tests/golden/force_reading_d2q9_128x64_theta60.json: the FP64
oracle's history of the D2Q9 128 x 64 sessile drop (8-node wall, R = 25,
tau = 1, M = 0.1, gamma = 2.5e-3, target 60 degrees) under the two forms of
the surface-tension force that Sec. II.B states: mu grad C (the form the
velocity moment carries, used throughout) and -C grad mu (as typeset).

Calls only the oracle (plus the seeded input generator and the angle fit).
Usage:  python tests/golden/make_force_reading_golden.py [steps]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2504_19941_amd import analysis as A  # noqa: E402
from paper_2504_19941_amd import workloads as W  # noqa: E402

EVERY = 5000
THETA = 60.0


def run(steps, threads=4):
    w = W.config_2d_contact_angle(THETA)
    sims = {}
    for name, fr in (("potential", O.FORCE_POTENTIAL), ("typeset", O.FORCE_AS_TYPESET)):
        o = O.Oracle(2, w.shape, w.kappa, mobility=w.mobility, tau=w.tau, threads=threads, force_reading=fr)
        o.set_solid_field(W.flat(w.C1))
        o.set_liquid(W.flat(w.C2))
        sims[name] = o
    hist = {k: [] for k in sims}
    for k in range(steps // EVERY):
        for name, o in sims.items():
            o.step(EVERY)
            fl = o.fields()
            u = fl["u"]
            th = A.contact_angle(W.unflat(fl["C1"], w.shape), W.unflat(fl["C2"], w.shape), 1, w.wall_level)
            hist[name].append({"step": (k + 1) * EVERY, "theta": th,
                               "umax": float(np.sqrt((u ** 2).sum(axis=0)).max()),
                               "C2max": float(fl["C2"].max())})
        print((k + 1) * EVERY, {n: (round(h[-1]["theta"], 3), h[-1]["umax"]) for n, h in hist.items()}, flush=True)
    return {"theta_target": THETA, "kappa": list(w.kappa), "every": EVERY, "history": hist,
            "about": ("FP64 oracle, D2Q9 128x64 periodic, wall rows y<=7 (analytic tanh, face y=7.5), "
                      "semicircular drop R=25 at x=64, tau=1, M=0.1, gamma=2.5e-3, theta 60; surface-tension "
                      "force mu grad C ('potential') and -C grad mu ('typeset'); written by "
                      "tests/golden/make_force_reading_golden.py")}


if __name__ == "__main__":
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 150000
    data = run(steps)
    json.dump(data, open(os.path.join(HERE, "force_reading_d2q9_128x64_theta60.json"), "w"), indent=1)
