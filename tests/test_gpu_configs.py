"""The workloads at their full sizes, in the launch configuration the
benchmark uses, against the FP64 oracle: the 256 x 256 x 192 micropillar
array (every node after a few steps, FP32 and FP16 storage), its cropped
64 x 64 x 96 version over 1000 steps, and spot parity of sampled members of
the 512-lattice sinusoidal-wall batch stepped in one batched launch.  The
micropillar solid is the analytic diffuse field of the seeded pillar layout
(both sides get the same C1)."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2504_19941_amd import dsm
from paper_2504_19941_amd import workloads as W

from .conftest import f32

pytestmark = pytest.mark.gpu


def report(name, a, b):
    err = float(np.abs(np.asarray(a) - np.asarray(b)).max())
    print(f"  {name}: max abs err {err:.3e}", flush=True)
    return err


def test_pillars_full_size_matches_oracle(gpu):
    w = W.config_3d_pillars_analytic()
    C1, C2 = f32(W.flat(w.C1)), f32(W.flat(w.C2))
    orc = Oracle(3, w.shape, w.kappa, gravity=w.gravity, threads=16)
    orc.set_solid_field(C1)
    orc.set_liquid(C2)
    orc.step(6)
    fo = orc.fields()
    orc.close()
    for storage, tol_c, tol_u in ((dsm.DSM_STORAGE_FP32, 1e-6, 1e-7), (dsm.DSM_STORAGE_FP16, 2e-5, 2e-6)):
        sim = dsm.Simulation(3, w.shape, w.kappa, gravity=w.gravity, storage=storage)
        sim.set_solid_field(C1)
        sim.set_liquid(C2)
        m0 = sim.mass()
        sim.step(6)
        fg = sim.fields()
        print(f"  storage {storage}:", flush=True)
        assert report("C2 (256x256x192, 6 steps)", fg["C2"], fo["C2"]) < tol_c
        assert report("u", fg["u"], fo["u"]) < tol_u
        m1 = sim.mass()
        assert abs(m1[1] - m0[1]) / m0[1] < 1e-9
        sim.close()


def test_pillars_cropped_1000_steps(gpu):
    w = W.config_3d_pillars_analytic((64, 64, 96), liquid=(44, 80))
    C1, C2 = f32(W.flat(w.C1)), f32(W.flat(w.C2))
    sim = dsm.Simulation(3, w.shape, w.kappa, gravity=w.gravity, reduce_every=250)
    orc = Oracle(3, w.shape, w.kappa, gravity=w.gravity, threads=16)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_liquid(C2)
    m0 = sim.mass()
    for s in (sim, orc):
        s.step(1000)
    fg, fo = sim.fields(), orc.fields()
    assert report("C2 (64x64x96 pillars, 1000 steps)", fg["C2"], fo["C2"]) < 1e-5
    assert report("u", fg["u"], fo["u"]) < 1e-6
    m1 = sim.mass()
    assert abs(m1[1] - m0[1]) / m0[1] < 1e-9
    orc.close()


def test_sinusoid_batch_spot_parity(gpu):
    """All 512 lattices stepped together (tuned schedule); the 8 smallest
    checked against the oracle run alone."""
    ws = W.batch_2d_sinusoid(512)
    sims = []
    for w in ws:
        s = dsm.Simulation(2, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility, gravity=w.gravity)
        s.set_solid_field(f32(W.flat(w.C1)))
        s.set_liquid(f32(W.flat(w.C2)))
        s.step(1)
        sims.append(s)
    batch = dsm.Batch(sims)
    batch.tune()
    batch.step(200)
    picks = sorted(range(len(ws)), key=lambda k: ws[k].nodes)[:8]
    for k in picks:
        w = ws[k]
        orc = Oracle(2, w.shape, w.kappa, alpha=w.alpha, tau=w.tau, mobility=w.mobility, gravity=w.gravity,
                     threads=8)
        orc.set_solid_field(f32(W.flat(w.C1)))
        orc.set_liquid(f32(W.flat(w.C2)))
        orc.step(201)
        fg, fo = sims[k].fields(), orc.fields()
        assert report(f"member {k} {w.name}", fg["C2"], fo["C2"]) < 1e-5
        assert np.abs(fg["u"] - fo["u"]).max() < 1e-6
        orc.close()
    batch.close()
