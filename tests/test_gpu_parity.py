"""GPU parity: the HIP step through the C ABI against the FP64 oracle on the
same seeded inputs (inputs rounded to FP32 first, so both see identical
values).  Sizes span several workgroup tiles with ragged tails (3D tiles are
at most 128 x 8 columns, 2D tiles at most 256 columns, each marching 8-32
planes)."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2504_19941_amd import dsm
from paper_2504_19941_amd import workloads as W

from .conftest import f32
from .geometry import wall_and_particle

pytestmark = pytest.mark.gpu

KERNELS = [dsm.DSM_KERNEL_FUSED, dsm.DSM_KERNEL_SPLIT]
SHAPES = {2: (150, 37), 3: (37, 21, 19)}
KAPPA = W.kappas_for_angle(70.0)


def pair(dim, shape, kernel, gravity=(0.0, 0.0, 0.0), mobility=0.1, tau=1.0, kappa=KAPPA, mask=None,
         storage=dsm.DSM_STORAGE_FP32):
    sim = dsm.Simulation(dim, shape, kappa, tau=tau, mobility=mobility, gravity=gravity, mask=mask,
                         kernel=kernel, reduce_every=0, storage=storage)
    orc = Oracle(dim, shape, kappa, tau=tau, mobility=mobility, gravity=gravity, mask=mask, threads=4)
    return sim, orc


def report(name, a, b):
    err = np.abs(np.asarray(a) - np.asarray(b)).max()
    print(f"  {name}: max abs err {err:.3e}", flush=True)
    return err


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_one_step_from_random_state(gpu, dim, kernel):
    shape = SHAPES[dim]
    mask, C1, C2 = wall_and_particle(dim, shape, seed=11)
    C1 = f32(W.flat(C1))
    Q = 9 if dim == 2 else 19
    fs, gs = W.random_postcollision_state(Q, shape, C2, seed=12, amp=1e-3)
    fs, gs = f32(fs), f32(gs)
    grav = (1e-4, -2e-4, 0.0) if dim == 2 else (1e-4, -2e-4, 3e-4)
    sim, orc = pair(dim, shape, kernel, gravity=grav)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_postcollision(fs, gs)
        s.step(1)
    fg, fo = sim.fields(), orc.fields()
    assert report("C2", fg["C2"], fo["C2"]) < 2e-6
    assert report("u", fg["u"], fo["u"]) < 2e-6
    assert report("p", fg["p"], fo["p"]) < 2e-6
    pg, po = sim.get_populations(), orc.get_populations()
    assert report("f", pg[0], po[0]) < 2e-6
    assert report("g", pg[1], po[1]) < 2e-6
    assert report("mu", sim.chemical_potential(), orc.chemical_potential()) < 1e-7


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_steps_from_liquid(gpu, dim, kernel):
    """t = 0 initialisation (post-stream state) and 400 steps with walls,
    a curved particle and a body force."""
    shape = SHAPES[dim]
    mask, C1, C2 = wall_and_particle(dim, shape, seed=21)
    C1, C2 = f32(W.flat(C1)), f32(W.flat(C2))
    grav = (2e-5, 0.0, 0.0) if dim == 2 else (2e-5, 1e-5, 0.0)
    sim, orc = pair(dim, shape, kernel, gravity=grav)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_liquid(C2)
    m0 = sim.mass()
    for s in (sim, orc):
        s.step(400)
    fg, fo = sim.fields(), orc.fields()
    assert report("C2", fg["C2"], fo["C2"]) < 1e-5
    assert report("u", fg["u"], fo["u"]) < 1e-6
    m1 = sim.mass()
    assert abs(m1[1] - m0[1]) / m0[1] < 1e-6
    Fg, Eg = sim.free_energy()
    Fo, Eo = orc.free_energy()
    assert abs(Fg - Fo) / abs(Fo) < 1e-5
    assert abs(Eg - Eo) <= 1e-3 * abs(Eo) + 1e-12
    # selected fields: the same values, only those returned
    for which in (("C2",), ("C3",), ("C1", "u"), ("p",), "C2"):
        sel = sim.fields(which)
        names = (which,) if isinstance(which, str) else which
        assert set(sel) == set(names)
        for k in names:
            assert np.array_equal(sel[k], fg[k]), k
    # the same FP64 reduction through dsm_diagnostics, with the largest speed
    d = sim.diagnostics()
    assert np.array_equal(d["mass"], m1)
    assert d["free_energy"] == Fg and d["kinetic_energy"] == Eg
    speed_o = float(np.sqrt((fo["u"] ** 2).sum(axis=0)).max())
    print(f"  max speed: gpu {d['max_speed']:.6e}, oracle {speed_o:.6e}", flush=True)
    assert abs(d["max_speed"] - speed_o) <= 1e-3 * speed_o
    assert d["nonfinite_nodes"] == 0.0


@pytest.mark.parametrize("storage,bar", [(dsm.DSM_STORAGE_FP32, 1e-5), (dsm.DSM_STORAGE_FP16, 2e-3)])
@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_liquid_on_the_sharp_mask(gpu, dim, kernel, storage, bar):
    """A liquid set right after creation on the sharp solid C1 = 1[S], with no
    solid stage: the cut links of the sharp field, built at creation, against
    the oracle's bounce-back on the same field, 300 steps (FP16 population
    storage to its bar)."""
    shape = SHAPES[dim]
    mask, _, _ = wall_and_particle(dim, shape, seed=41)
    C1 = mask.astype(np.float64)
    centre = [0.6 * n for n in shape[:-1]] + [3.5]
    C2 = f32(W.flat(W.drop_field(shape, centre, 0.3 * min(shape), C1, open_axis=dim - 1)))
    grav = (2e-5, 0.0, 0.0) if dim == 2 else (2e-5, 1e-5, 0.0)
    sim, orc = pair(dim, shape, kernel, gravity=grav, mask=W.flat(mask), storage=storage)
    for s in (sim, orc):
        s.set_liquid(C2)
        s.step(300)
    fg, fo = sim.fields(), orc.fields()
    assert np.array_equal(fg["C1"], W.flat(C1))
    assert report("C2", fg["C2"], fo["C2"]) < bar
    assert report("u", fg["u"], fo["u"]) < bar / 10
    assert np.abs(fo["u"]).max() > 1e-6  # the flow is not trivial


@pytest.mark.parametrize("storage,bar", [(dsm.DSM_STORAGE_FP32, 1e-5), (dsm.DSM_STORAGE_FP16, 2e-3)])
@pytest.mark.parametrize("dim", [2, 3])
def test_solid_stage(gpu, dim, storage, bar):
    """Solid stage from the sharp mask (confinement and range penalty on),
    1000 steps in two calls with different beta and Omega, then the frozen C1
    against the oracle; with FP16 population storage to the FP16 bar."""
    shape = SHAPES[dim]
    mask, _, _ = wall_and_particle(dim, shape, seed=31)
    m = W.flat(mask)
    k = W.kappas_for_angle(90.0)
    sim, orc = pair(dim, shape, dsm.DSM_KERNEL_FUSED, kappa=k, mask=m, storage=storage)
    for s in (sim, orc):
        s.init_solid(300, 1e-2, 1e-2, 1.0, 1.0 / 6.0, dsm.DSM_SOLID_RESET)
        s.init_solid(700, 1e-3, 2e-4, 1.0, 1.0 / 6.0, 0)
    fg, fo = sim.fields(), orc.fields()
    assert report("C1", fg["C1"], fo["C1"]) < bar
    assert np.array_equal(sim.fields(("C1",))["C1"], fg["C1"])
    assert np.array_equal(sim.fields(("C3",))["C3"], fg["C3"])


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_one_node_slit_bounce_back_fallback(gpu, dim, kernel):
    """A fluid slit one node wide between two diffuse slabs (off-centre):
    every cut link of the slit takes the q < 1/2 fallback to halfway
    bounce-back or has q = 1/2 already, so sum f over the fluid nodes is
    conserved; the GPU follows the oracle node by node over 40 steps."""
    from oracle.oracle import lattice

    shape = (150, 9) if dim == 2 else (37, 21, 9)
    coords = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    dz = np.abs(coords[-1] - 4.2)
    C1 = f32(W.flat(W.tanh_profile(np.minimum(dz, shape[-1] - dz) - 0.5)))
    fluid = C1 < 0.5
    Q, N = (9, 19)[dim - 2], C1.size
    _, w = lattice(dim)
    rng = np.random.default_rng(43)
    fs = f32(np.asarray(w)[:, None] * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=(Q, N))) * fluid)
    gs = np.zeros((Q, N))
    gs[0] = 0.3 * fluid
    sim, orc = pair(dim, shape, kernel, kappa=W.kappas_for_angle(90.0), tau=0.8)
    for s in (sim, orc):
        s.set_solid_field(C1)
        s.set_postcollision(fs, gs)
        s.step(40)
    s0 = fs[:, fluid].sum()
    pg, po = sim.get_populations(), orc.get_populations()
    drift = abs(pg[0][:, fluid].sum() - s0) / s0
    print(f"  sum f over the slit: relative drift {drift:.2e} (oracle "
          f"{abs(po[0][:, fluid].sum() - s0) / s0:.2e})", flush=True)
    assert drift < 1e-5
    assert report("f", pg[0][:, fluid], po[0][:, fluid]) < 2e-6
    fg, fo = sim.fields(), orc.fields()
    assert report("u", fg["u"][:, fluid], fo["u"][:, fluid]) < 2e-6


def test_fused_matches_split(gpu):
    shape = (64, 40, 36)
    mask, C1, C2 = wall_and_particle(3, shape, seed=41)
    res = []
    for kernel in KERNELS:
        sim = dsm.Simulation(3, shape, KAPPA, kernel=kernel)
        sim.set_solid_field(W.flat(C1))
        sim.set_liquid(W.flat(C2))
        sim.step(200)
        res.append(sim.fields())
    assert report("C2", res[0]["C2"], res[1]["C2"]) < 1e-6
    assert report("u", res[0]["u"], res[1]["u"]) < 1e-7


def test_deterministic(gpu):
    shape = (48, 40, 33)
    mask, C1, C2 = wall_and_particle(3, shape, seed=51)
    states = []
    for _ in range(2):
        sim = dsm.Simulation(3, shape, KAPPA)
        sim.set_solid_field(W.flat(C1))
        sim.set_liquid(W.flat(C2))
        sim.step(50)
        states.append(sim.get_state())
    assert states[0] == states[1]
