"""GPU acceptance against the FP64 oracle at the bars the method is held to:
per-node concentration within 1e-5 after 1000 FP32 steps, liquid mass drift
below 1e-6 relative, equilibrium contact angles within 0.5 degrees of the
oracle's (and near Young's law), the full 128^3 lattice in the launch
configuration the benchmark times, invariance of results under the launch
shape, checkpoint/resume, the degenerate cases, and the instability check.

Inputs are seeded and rounded to FP32 before both sides see them."""
import json
import os

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2504_19941_amd import analysis as A
from paper_2504_19941_amd import dsm
from paper_2504_19941_amd import workloads as W

from .conftest import f32
from .geometry import wall_and_particle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KAPPA = W.kappas_for_angle(70.0)


def report(name, a, b):
    err = float(np.abs(np.asarray(a) - np.asarray(b)).max())
    print(f"  {name}: max abs err {err:.3e}", flush=True)
    return err


# shapes spanning several workgroup tiles with ragged tails on every axis
# (the default 3D tile is 128 x 4 columns, the 2D tile 256 columns; marches of
# 8-32 planes)
SHAPES_1000 = [(2, (300, 37)), (3, (40, 21, 35)), (3, (130, 9, 18))]


@pytest.mark.parametrize("dim,shape", SHAPES_1000)
def test_1000_steps_match_oracle(gpu, dim, shape):
    mask, C1, C2 = wall_and_particle(dim, shape, seed=61)
    C1, C2 = f32(W.flat(C1)), f32(W.flat(C2))
    grav = (1e-5, -2e-6, 0.0) if dim == 2 else (1e-5, 3e-6, -2e-6)
    sim = dsm.Simulation(dim, shape, KAPPA, gravity=grav, reduce_every=250)
    orc = Oracle(dim, shape, KAPPA, gravity=grav, threads=8)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_liquid(C2)
    m0 = sim.mass()
    for s in (sim, orc):
        s.step(1000)
    fg, fo = sim.fields(), orc.fields()
    assert report("C2", fg["C2"], fo["C2"]) < 1e-5
    assert report("C3", fg["C3"], fo["C3"]) < 1e-5
    assert report("u", fg["u"], fo["u"]) < 1e-6
    m1 = sim.mass()
    drift = abs(m1[1] - m0[1]) / m0[1]
    print(f"  liquid mass drift {drift:.2e}", flush=True)
    assert drift < 1e-9
    mo = orc.mass()
    assert abs(m1[1] - mo[1]) / mo[1] < 1e-6


def test_full_size_lattice_in_bench_configuration(gpu):
    """The benchmark's 128^3 sessile drop, default launch shape: every node
    against the oracle after 8 steps, and the mirror symmetry of the drop
    (centred on x = y = 64) after 300 steps."""
    w = W.config_3d_sessile(90.0, n=128)
    C1, C2 = f32(W.flat(w.C1)), f32(W.flat(w.C2))
    sim = dsm.Simulation(3, w.shape, w.kappa, tau=w.tau, mobility=w.mobility)
    orc = Oracle(3, w.shape, w.kappa, tau=w.tau, mobility=w.mobility, threads=16)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_liquid(C2)
        s.step(8)
    fg, fo = sim.fields(), orc.fields()
    assert report("C2 (128^3, 8 steps)", fg["C2"], fo["C2"]) < 1e-6
    assert report("u (128^3, 8 steps)", fg["u"], fo["u"]) < 1e-7
    orc.close()
    sim.step(292)
    fl = sim.fields()
    C2g = W.unflat(fl["C2"], w.shape)
    idx = (128 - np.arange(128)) % 128
    assert report("mirror x", C2g, C2g[idx]) < 1e-6
    assert report("mirror y", C2g, C2g[:, idx]) < 1e-6


def test_default_tiling_and_its_readback(gpu):
    """dsm_get_tiling reports the launch shape in use: the default dsm_create
    chose, then whatever dsm_set_tiling set.  On a 256-CU MI355X the defaults
    of the benchmark-type lattices are the measured best ones: 128x4 tiles
    marching 16 planes for the 128^3 FP32 lattice and 8 with FP16 storage;
    96 planes (FP32) and 48 (FP16) for the 256 x 256 x 192 pillar lattice,
    one round of tiles each; 8 planes for an 80^3 FP32 lattice, too small
    to fill the chip with 16;
    64-column tiles with 8-row marches for a D2Q9 lattice 300 columns wide;
    1-row marches on 128-column tiles for D2Q9 128 x 64 and 4-row marches
    on 128-column tiles for 100 x 4096, whose default grids fill at most half
    a round; 2-plane marches on 64-column tiles for a 64^3 lattice, likewise."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cases = [(3, (128, 128, 128), dsm.DSM_STORAGE_FP32, (2, 16)),
             (3, (128, 128, 128), dsm.DSM_STORAGE_FP16, (2, 8)),
             (3, (256, 256, 192), dsm.DSM_STORAGE_FP32, (2, 96)),
             (3, (256, 256, 192), dsm.DSM_STORAGE_FP16, (2, 48)),
             (3, (80, 80, 80), dsm.DSM_STORAGE_FP32, (2, 8)),
             (2, (300, 8192), dsm.DSM_STORAGE_FP32, (2, 8)),
             (2, (128, 64), dsm.DSM_STORAGE_FP32, (1, 1)),
             (2, (100, 4096), dsm.DSM_STORAGE_FP16, (1, 4)),
             (3, (64, 64, 64), dsm.DSM_STORAGE_FP32, (0, 2)),
             (3, (64, 64, 64), dsm.DSM_STORAGE_FP16, (0, 2))]
    for dim, shape, storage, expect in cases:
        sim = dsm.Simulation(dim, shape, KAPPA, storage=storage)
        variant, planes = sim.tiling()
        assert 0 <= variant < dsm.dsm_tiling_variants(dim) and planes in (1, 2, 4, 8, 16, 32, 48, 64, 96, 128)
        if cus == 256:
            assert (variant, planes) == expect, (shape, storage, (variant, planes))
        sim.set_tiling(0, 12)
        assert sim.tiling() == (0, 12)
        sim.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_launch_shape_does_not_change_results(gpu, dim):
    """Every tile variant and march length computes bit-identical states."""
    shape = (150, 37) if dim == 2 else (70, 13, 21)
    mask, C1, C2 = wall_and_particle(dim, shape, seed=71)
    ref = None
    for variant in range(dsm.dsm_tiling_variants(dim)):
        for planes in (1, 3, 16, 64):
            sim = dsm.Simulation(dim, shape, KAPPA, gravity=(1e-5, 0.0, 0.0))
            sim.set_tiling(variant, planes)
            sim.set_solid_field(W.flat(C1))
            sim.set_liquid(W.flat(C2))
            sim.step(30)
            st = sim.get_state()
            if ref is None:
                ref = st
            assert st == ref, f"variant {variant} planes {planes} differs"


@pytest.mark.parametrize("dim,shape", [(2, (300, 120)), (3, (96, 40, 50))])
def test_measured_tiling_tuner(gpu, dim, shape):
    """dsm_tune_tiling times every variant and march on the lattice itself,
    installs one of them, and leaves the state where the same number of
    plain steps leaves it (the tiling changes no result)."""
    mask, C1, C2 = wall_and_particle(dim, shape, seed=73)
    sims = []
    for _ in range(2):
        sim = dsm.Simulation(dim, shape, KAPPA, gravity=(1e-5, 0.0, 0.0))
        sim.set_solid_field(W.flat(C1))
        sim.set_liquid(W.flat(C2))
        sims.append(sim)
    tuned, plain = sims
    v, planes, ms = tuned.tune_tiling(reps=2)
    taken = tuned.steps
    print(f"  tuned tiling ({v}, {planes}), fused kernel {ms * 1e3:.1f} us, {taken} steps taken", flush=True)
    assert 0 <= v < dsm.dsm_tiling_variants(dim) and planes >= 1 and ms > 0.0
    assert tuned.tiling() == (v, planes)
    assert taken >= dsm.dsm_tiling_variants(dim) * 3
    plain.step(taken)
    assert tuned.get_state() == plain.get_state()
    tuned.step(5)
    plain.step(5)
    assert tuned.get_state() == plain.get_state()
    with pytest.raises(dsm.DsmError):
        dsm.dsm_tune_tiling(tuned.handle, 0)


def test_checkpoint_resume_is_bitwise(gpu):
    shape = (48, 20, 24)
    mask, C1, C2 = wall_and_particle(3, shape, seed=81)
    a = dsm.Simulation(3, shape, KAPPA, gravity=(0.0, 1e-5, 0.0))
    a.set_solid_field(W.flat(C1))
    a.set_liquid(W.flat(C2))
    a.step(57)
    saved = a.get_state()
    a.step(60)
    b = dsm.Simulation(3, shape, KAPPA, gravity=(0.0, 0.0, 0.0))
    b.set_state(saved)
    assert b.steps == 57
    b.step(60)
    assert a.get_state() == b.get_state()


@pytest.mark.parametrize("dim,shape", [(2, (4, 4)), (3, (4, 4, 4)), (2, (5, 300)), (3, (67, 5, 4))])
def test_smallest_and_thin_lattices(gpu, dim, shape):
    """Lattices narrower than one wave, one tile or one march."""
    rng = np.random.default_rng(5)
    N = int(np.prod(shape))
    C1 = f32(np.where(rng.uniform(size=N) < 0.06, 0.9, 0.05))
    C2 = f32(rng.uniform(0.0, 0.6, N) * (1.0 - C1))
    sim = dsm.Simulation(dim, shape, KAPPA, mobility=0.05)
    orc = Oracle(dim, shape, KAPPA, mobility=0.05)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_liquid(C2)
        s.step(40)
    fg, fo = sim.fields(), orc.fields()
    assert report("C2", fg["C2"], fo["C2"]) < 1e-5
    assert report("u", fg["u"], fo["u"]) < 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_liquid_and_empty_liquid_are_fixed_points(gpu, dim):
    shape = (70, 9) if dim == 2 else (20, 9, 11)
    N = int(np.prod(shape))
    for level in (0.0, 0.37):
        sim = dsm.Simulation(dim, shape, KAPPA)
        sim.set_solid_field(np.zeros(N))
        sim.set_liquid(np.full(N, f32(level)))
        sim.step(100)
        fl = sim.fields()
        assert np.abs(fl["C2"] - f32(level)).max() < 1e-6
        assert np.abs(fl["u"]).max() < 1e-9


def test_instability_is_reported(gpu):
    """A body force far beyond the scheme's range drives the state to
    non-finite values; the periodic check reports DSM_EUNSTABLE."""
    shape = (64, 16)
    mask, C1, C2 = wall_and_particle(2, shape, seed=91)
    sim = dsm.Simulation(2, shape, KAPPA, gravity=(50.0, 0.0, 0.0), reduce_every=50)
    sim.set_solid_field(W.flat(C1))
    sim.set_liquid(W.flat(C2))
    with pytest.raises(dsm.DsmError) as e:
        sim.step(2000)
    assert e.value.code == dsm.DSM_EUNSTABLE


def _golden(theta):
    path = os.path.join(GOLDEN, f"young_d2q9_128x64_theta{theta:g}.json")
    if not os.path.exists(path):
        pytest.skip(f"missing {path}")
    return json.load(open(path))


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0])
def test_contact_angle_matches_oracle_and_young(gpu, theta):
    """D2Q9 128 x 64 sessile drop (8-node wall, R = 25): the FP32 GPU angle
    follows the FP64 oracle's within 0.5 degrees at 20k steps (the run length
    of this workload) and at the end of the stored history, and the final
    angle is within 2 degrees of Young's law (eqn:st_ca)."""
    gold = _golden(theta)
    hist = {h["step"]: h["theta"] for h in gold["history"]}
    w = W.config_2d_contact_angle(theta)
    sim = dsm.Simulation(2, w.shape, w.kappa, tau=w.tau, mobility=w.mobility, reduce_every=10000)
    sim.set_solid_field(f32(W.flat(w.C1)))
    sim.set_liquid(f32(W.flat(w.C2)))
    m0 = sim.mass()
    done = 0
    checks = [20000, max(hist)]
    for target in checks:
        sim.step(target - done)
        done = target
        fl = sim.fields()
        th = A.contact_angle(W.unflat(fl["C1"], w.shape), W.unflat(fl["C2"], w.shape), 1, w.wall_level)
        print(f"  theta {theta}: step {target}: gpu {th:.3f}, oracle {hist[target]:.3f}", flush=True)
        assert abs(th - hist[target]) < 0.5
    assert abs(th - theta) < 2.0
    drift = abs(sim.mass()[1] - m0[1]) / m0[1]
    print(f"  liquid mass drift after {done} steps: {drift:.2e}", flush=True)
    assert drift < 1e-9


# --- FP16 population storage -------------------------------------------------

@pytest.mark.parametrize("dim,shape", SHAPES_1000)
def test_fp16_storage_1000_steps(gpu, dim, shape):
    """Populations stored as FP16 (FP32 arithmetic): concentrations within
    2e-3 of the FP64 oracle after 1000 steps, and the liquid mass conserved
    (the FP64 rest population absorbs the rounding of the moving ones)."""
    mask, C1, C2 = wall_and_particle(dim, shape, seed=61)
    C1, C2 = f32(W.flat(C1)), f32(W.flat(C2))
    grav = (1e-5, -2e-6, 0.0) if dim == 2 else (1e-5, 3e-6, -2e-6)
    sim = dsm.Simulation(dim, shape, KAPPA, gravity=grav, storage=dsm.DSM_STORAGE_FP16)
    orc = Oracle(dim, shape, KAPPA, gravity=grav, threads=8)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_liquid(C2)
    m0 = sim.mass()
    for s in (sim, orc):
        s.step(1000)
    fg, fo = sim.fields(), orc.fields()
    assert report("C2 (fp16 storage)", fg["C2"], fo["C2"]) < 2e-3
    assert report("u (fp16 storage)", fg["u"], fo["u"]) < 1e-4
    drift = abs(sim.mass()[1] - m0[1]) / m0[1]
    print(f"  liquid mass drift {drift:.2e}", flush=True)
    assert drift < 1e-9


def test_fp16_launch_shape_does_not_change_results(gpu):
    shape = (70, 13, 21)
    mask, C1, C2 = wall_and_particle(3, shape, seed=71)
    ref = None
    for variant in range(dsm.dsm_tiling_variants(3)):
        for planes in (1, 16):
            sim = dsm.Simulation(3, shape, KAPPA, gravity=(1e-5, 0.0, 0.0), storage=dsm.DSM_STORAGE_FP16)
            sim.set_tiling(variant, planes)
            sim.set_solid_field(W.flat(C1))
            sim.set_liquid(W.flat(C2))
            sim.step(30)
            st = sim.get_state()
            if ref is None:
                ref = st
            assert st == ref, f"variant {variant} planes {planes} differs"


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0])
def test_fp16_contact_angle(gpu, theta):
    """FP16 storage: the equilibrium angle within 1 degree of the FP64
    oracle's, at 20k steps and at the end of the stored history."""
    gold = _golden(theta)
    hist = {h["step"]: h["theta"] for h in gold["history"]}
    w = W.config_2d_contact_angle(theta)
    sim = dsm.Simulation(2, w.shape, w.kappa, tau=w.tau, mobility=w.mobility, reduce_every=10000,
                         storage=dsm.DSM_STORAGE_FP16)
    sim.set_solid_field(f32(W.flat(w.C1)))
    sim.set_liquid(f32(W.flat(w.C2)))
    done = 0
    for target in [20000, max(hist)]:
        sim.step(target - done)
        done = target
        fl = sim.fields()
        th = A.contact_angle(W.unflat(fl["C1"], w.shape), W.unflat(fl["C2"], w.shape), 1, w.wall_level)
        print(f"  fp16 theta {theta}: step {target}: gpu {th:.3f}, oracle {hist[target]:.3f}", flush=True)
        assert abs(th - hist[target]) < 1.0
