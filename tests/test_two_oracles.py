"""The C oracle and the independent NumPy oracle agree to round-off on small
lattices, in both stages, with walls, a curved particle, interpolated
bounce-back, a body force, and density and viscosity contrast."""
import numpy as np
import pytest

from oracle.mini_oracle import MiniOracle, lattice
from oracle.oracle import Oracle
from oracle.oracle import lattice as c_lattice
from paper_2504_19941_amd import workloads as W

from .geometry import wall_and_particle

CASES = [(2, (16, 16)), (3, (8, 8, 8)), (3, (10, 9, 8))]


@pytest.mark.parametrize("dim", [2, 3])
def test_same_lattice(oracle_lib, dim):
    c, w = lattice(dim)
    c2, w2 = c_lattice(dim)
    assert np.array_equal(c, c2[:, :dim])
    assert np.allclose(w, w2, rtol=0, atol=1e-17)


@pytest.mark.parametrize("dim,shape", CASES)
def test_fluid_stage(oracle_lib, dim, shape):
    mask, C1, C2 = wall_and_particle(dim, shape, thickness=2, radius=2.5, seed=3)
    k = W.kappas_for_angle(70.0)
    grav = (1e-4, -2e-4, 3e-4)[:dim] + (0.0,) * (3 - dim)
    o = Oracle(dim, shape, k, gravity=grav, mask=W.flat(mask))
    m = MiniOracle(dim, shape, k, gravity=grav, mask=mask)
    o.set_solid_field(W.flat(C1))
    m.set_solid_field(C1)
    o.set_liquid(W.flat(C2))
    m.set_liquid(C2)
    o.step(100)
    m.step(100)
    fo, fm = o.fields(), m.fields()
    for key in ("C2", "p"):
        assert np.abs(fo[key] - fm[key]).max() < 1e-13
    assert np.abs(fo["u"] - fm["u"]).max() < 1e-13
    po, pm = o.get_populations(), m.populations()
    assert np.abs(po[0] - pm[0]).max() < 1e-13
    assert np.abs(po[1] - pm[1]).max() < 1e-13


@pytest.mark.parametrize("dim,shape", CASES)
def test_fluid_stage_on_the_sharp_mask(oracle_lib, dim, shape):
    """A liquid set right after creation, on the sharp solid C1 = 1[S] (no
    solid stage): bounce-back with the wall fractions of the sharp field."""
    mask, _, _ = wall_and_particle(dim, shape, thickness=2, radius=2.5, seed=8)
    C1 = mask.astype(np.float64)
    C2 = W.drop_field(shape, [0.7 * n for n in shape[:-1]] + [1.5], 0.3 * min(shape), C1, open_axis=dim - 1)
    k = W.kappas_for_angle(70.0)
    grav = (1e-4, -2e-4, 3e-4)[:dim] + (0.0,) * (3 - dim)
    o = Oracle(dim, shape, k, gravity=grav, mask=W.flat(mask))
    m = MiniOracle(dim, shape, k, gravity=grav, mask=mask)
    o.set_liquid(W.flat(C2))
    m.set_liquid(C2)
    o.step(100)
    m.step(100)
    fo, fm = o.fields(), m.fields()
    assert np.array_equal(fo["C1"], W.flat(C1))
    for key in ("C2", "p"):
        assert np.abs(fo[key] - fm[key]).max() < 1e-13
    assert np.abs(fo["u"] - fm["u"]).max() < 1e-13
    assert np.abs(fo["u"]).max() > 1e-6


@pytest.mark.parametrize("dim,shape", CASES)
def test_solid_stage(oracle_lib, dim, shape):
    mask, _, _ = wall_and_particle(dim, shape, thickness=2, radius=2.5, seed=4)
    k = W.kappas_for_angle(90.0)
    o = Oracle(dim, shape, k, mask=W.flat(mask))
    m = MiniOracle(dim, shape, k, mask=mask)
    o.init_solid(60, 1e-2, 1e-2)
    m.init_solid(60, 1e-2, 1e-2)
    o.init_solid(40, 1e-3, 2e-4, flags=0)
    m.init_solid(40, 1e-3, 2e-4, reset=False)
    assert np.abs(o.fields()["C1"] - m.fields()["C1"]).max() < 1e-13


@pytest.mark.parametrize("dim,shape", [(2, (16, 16)), (3, (8, 8, 8))])
def test_random_postcollision_state(oracle_lib, dim, shape):
    mask, C1, C2 = wall_and_particle(dim, shape, thickness=2, radius=2.5, seed=6)
    Q = 9 if dim == 2 else 19
    fs, gs = W.random_postcollision_state(Q, shape, C2, seed=7)
    k = W.kappas_for_angle(50.0)
    o = Oracle(dim, shape, k)
    m = MiniOracle(dim, shape, k)
    o.set_solid_field(W.flat(C1))
    m.set_solid_field(C1)
    o.set_postcollision(fs, gs)
    m.set_postcollision(fs, gs)
    o.step(3)
    m.step(3)
    po, pm = o.get_populations(), m.populations()
    assert np.abs(po[0] - pm[0]).max() < 1e-13
    assert np.abs(po[1] - pm[1]).max() < 1e-13


@pytest.mark.parametrize("dim,shape", CASES)
def test_fluid_stage_with_density_and_viscosity_contrast(oracle_lib, dim, shape):
    mask, C1, C2 = wall_and_particle(dim, shape, thickness=2, radius=2.5, seed=5)
    k = W.kappas_for_angle(60.0)
    grav = (2e-4, -1e-4, 1e-4)[:dim] + (0.0,) * (3 - dim)
    kw = dict(gravity=grav, rho=(1.0, 0.4), tau_gas=0.62)
    o = Oracle(dim, shape, k, mask=W.flat(mask), **kw)
    m = MiniOracle(dim, shape, k, mask=mask, **kw)
    o.set_solid_field(W.flat(C1))
    m.set_solid_field(C1)
    o.set_liquid(W.flat(C2))
    m.set_liquid(C2)
    o.step(100)
    m.step(100)
    fo, fm = o.fields(), m.fields()
    for key in ("C2", "p"):
        assert np.abs(fo[key] - fm[key]).max() < 1e-13
    assert np.abs(fo["u"] - fm["u"]).max() < 1e-13
    assert np.abs(fo["u"]).max() > 1e-6  # the flow is not trivial
    po, pm = o.get_populations(), m.populations()
    assert np.abs(po[0] - pm[0]).max() < 1e-13
    assert np.abs(po[1] - pm[1]).max() < 1e-13
