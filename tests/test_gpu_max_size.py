"""The largest lattices the boundary accepts: 580^3 D3Q19 (195 million
nodes, 4.1e9 population slots against the limit of 2^32 - 1; 75 GiB of
device memory with FP32 populations), with FP32 and with FP16 storage.  No FP64 run of the whole lattice is
possible, but a state that varies along one axis only evolves exactly as the
same profile does on a lattice 4 nodes wide in the other two (the scheme is
local and translation invariant, and periodic in every axis), so the FP64
oracle runs that thin lattice and the GPU's fields are compared at every node
of sampled columns spread over the whole lattice, including its last rows and
planes, where the largest offsets are formed:

* along z (the slowest axis, the largest plane offsets): a diffuse solid
  slab and a liquid slab above it, 40 steps (bounce-back at the solid);
* along x (the fastest axis): a liquid column varying along x, no solid,
  20 steps.

Inputs are rounded to FP32 first, as in the other parity tests; the bars
are those of the other parity tests for each storage."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2504_19941_amd import dsm
from paper_2504_19941_amd import workloads as W

from .conftest import f32

pytestmark = pytest.mark.gpu

N = 580
KAPPA = W.kappas_for_angle(75.0)


def report(name, a, b):
    err = float(np.abs(np.asarray(a) - np.asarray(b)).max())
    print(f"  {name}: max abs err {err:.3e}", flush=True)
    return err


def profiles(axis):
    """C1, C2 of the profile along `axis` on a line of N nodes."""
    s = np.arange(N, dtype=np.float64)
    if axis == 2:
        C1 = W.tanh_profile(W.periodic_slab_distance(s, -0.5, 7.5, N))
        C2 = W.tanh_profile(W.periodic_slab_distance(s, 7.5, 300.0, N)) * (1.0 - C1)
    else:
        C1 = np.zeros(N)
        C2 = 0.5 + 0.4 * np.sin(2.0 * np.pi * 3.0 * s / N) * np.tanh((s - 0.3 * N) / 20.0)
    return f32(C1), f32(C2)


def thin_oracle(axis, C1, C2, steps, gravity):
    shape = [4, 4, 4]
    shape[axis] = N
    orc = Oracle(3, tuple(shape), KAPPA, gravity=gravity, threads=16)
    X = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")[axis]
    orc.set_solid_field(W.flat(C1[X]))
    orc.set_liquid(W.flat(C2[X]))
    orc.step(steps)
    fo = orc.fields()
    orc.close()
    idx = np.arange(N) * (1 if axis == 0 else 16)  # the line x = 0, y = 0 (x fastest)
    return {"C2": fo["C2"][idx], "u": fo["u"][:, idx]}


@pytest.mark.parametrize("storage,bar_c,bar_u", [(dsm.DSM_STORAGE_FP32, 1e-6, 1e-7),
                                                 (dsm.DSM_STORAGE_FP16, 2e-3, 1e-4)])
def test_largest_lattice_matches_thin_oracle(gpu, storage, bar_c, bar_u):
    shape = (N, N, N)
    sim = dsm.Simulation(3, shape, KAPPA, reduce_every=0, storage=storage)
    print(f"  {shape}: {N ** 3} nodes, device buffer {sim.nbytes / 2 ** 30:.1f} GiB, tiling {sim.tiling()}",
          flush=True)
    rng = np.random.default_rng(13)
    cols = [(0, 0), (N - 1, N - 1), (N - 1, 0), (0, N - 1)] + [tuple(rng.integers(0, N, 2)) for _ in range(8)]
    for axis, steps, gravity in ((2, 40, (0.0, 0.0, -1e-5)), (0, 20, (0.0, 0.0, 0.0))):
        C1, C2 = profiles(axis)
        sim.set_gravity(gravity)
        shape3 = [1, 1, 1]
        shape3[axis] = N
        full = lambda a: np.broadcast_to(a.reshape(shape3), shape).reshape(-1, order="F")  # noqa: E731
        sim.set_solid_field(full(C1))
        sim.set_liquid(full(C2))
        m0 = sim.mass()
        sim.step(steps)
        fg = sim.fields()
        ref = thin_oracle(axis, C1, C2, steps, gravity)
        print(f"  profile along axis {axis}, {steps} steps:", flush=True)
        C2g = W.unflat(fg["C2"], shape)
        u = [W.unflat(fg["u"][k], shape) for k in range(3)]
        for a, b in cols:
            if axis == 2:
                line_c, line_u = C2g[a, b, :], np.stack([u[k][a, b, :] for k in range(3)])
            else:
                line_c, line_u = C2g[:, a, b], np.stack([u[k][:, a, b] for k in range(3)])
            assert np.abs(line_c - ref["C2"]).max() < bar_c, (axis, a, b)
            assert np.abs(line_u - ref["u"]).max() < bar_u, (axis, a, b)
        report(f"C2 on {len(cols)} columns", np.stack([C2g[a, b, :] if axis == 2 else C2g[:, a, b] for a, b in cols]),
               np.broadcast_to(ref["C2"], (len(cols), N)))
        # and the whole lattice is still one profile: every column equals the first
        if axis == 2:
            spread = float(np.abs(C2g - C2g[:1, :1, :]).max())
        else:
            spread = float(np.abs(C2g - C2g[:, :1, :1]).max())
        print(f"  largest departure of any node from its column profile: {spread:.2e}", flush=True)
        assert spread == 0.0
        m1 = sim.mass()
        assert abs(m1[1] - m0[1]) / m0[1] < 1e-9
        del fg, C2g, u
    sim.close()
