"""dsm_diagnostics_noalloc, the entry point for callers that cannot allocate
device memory, against dsm_diagnostics on the same handles: two calls in a
row, the second on a smaller lattice (so a stale partial row of the first
call would show), each bit-identical to the allocating form's result."""
import numpy as np
import pytest

from paper_2504_19941_amd import dsm
from paper_2504_19941_amd import workloads as W

from .conftest import f32
from .geometry import wall_and_particle

pytestmark = pytest.mark.gpu


def stepped(dim, shape, steps, seed):
    _, C1, C2 = wall_and_particle(dim, shape, seed=seed)
    grav = (2e-5, 0.0, 0.0) if dim == 2 else (2e-5, 1e-5, 0.0)
    sim = dsm.Simulation(dim, shape, W.kappas_for_angle(70.0), gravity=grav)
    sim.set_solid_field(f32(W.flat(C1)))
    sim.set_liquid(f32(W.flat(C2)))
    sim.step(steps)
    return sim


def test_noalloc_diagnostics_match_the_allocating_form(gpu):
    big = stepped(3, (160, 48, 40), 120, seed=81)     # 1200 blocks of 256 nodes: the grid caps at 1024
    small = stepped(2, (37, 19), 60, seed=83)          # 3 reduction blocks
    for sim in (big, small):
        got = dsm.dsm_diagnostics_noalloc(sim.handle)
        want = sim.diagnostics()
        print(f"  {sim.shape}: mass {got['mass']}, F {got['free_energy']:.9e}, "
              f"max speed {got['max_speed']:.3e}", flush=True)
        assert np.array_equal(got["mass"], want["mass"])
        for k in ("free_energy", "kinetic_energy", "max_speed", "nonfinite_nodes"):
            assert got[k] == want[k], k
        assert want["max_speed"] > 0.0
    # and again, now that the array holds the small lattice's rows
    again = dsm.dsm_diagnostics_noalloc(big.handle)
    assert np.array_equal(again["mass"], big.diagnostics()["mass"])
    assert again["free_energy"] == big.diagnostics()["free_energy"]
