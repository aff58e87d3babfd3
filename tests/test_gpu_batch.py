"""Batched form on the GPU: each member of a batch of uneven 2D and 3D
lattices advances exactly (bit for bit) as it does alone under dsm_step,
whatever the schedule; the modelled tuner leaves the state untouched, the
measured one advances it as single steps would; a member
checked against the FP64 oracle directly; the error paths of the batch
calls."""
import ctypes

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2504_19941_amd import dsm
from paper_2504_19941_amd import workloads as W

from .conftest import f32
from .geometry import wall_and_particle

pytestmark = pytest.mark.gpu

# uneven members: ragged tails against every tile shape, several per type
SPECS = [(2, (100, 37)), (2, (64, 32)), (2, (300, 45)), (2, (129, 70)),
         (3, (40, 21, 35)), (3, (70, 20, 18)), (3, (33, 9, 12))]


def member_inputs(k, dim, shape):
    if dim == 2:
        rng = np.random.default_rng(500 + k)
        amp = float(rng.uniform(2.0, 6.0))
        lam = shape[0] / max(1, round(shape[0] / float(rng.uniform(16.0, 64.0))))
        mask, C1 = W.sinusoid_surface(shape, amp, lam, amp + 4.0)
        C2 = W.drop_field(shape, (0.5 * shape[0], amp + 4.0), min(12.0, 0.3 * shape[1]), C1, open_axis=1)
        theta = 50.0 + 12.0 * k
        grav = (10.0 ** (-7 + 0.5 * k), 0.0, 0.0)
    else:
        mask, C1, C2 = wall_and_particle(dim, shape, seed=600 + k)
        theta = 70.0 + 10.0 * k
        grav = (1e-5, 3e-6, -2e-6)
    return W.kappas_for_angle(theta), grav, f32(W.flat(C1)), f32(W.flat(C2))


def make_members(specs, storage=dsm.DSM_STORAGE_FP32, first_step=True):
    sims = []
    for k, (dim, shape) in enumerate(specs):
        kappa, grav, C1, C2 = member_inputs(k, dim, shape)
        s = dsm.Simulation(dim, shape, kappa, gravity=grav, storage=storage)
        s.set_solid_field(C1)
        s.set_liquid(C2)
        if first_step:
            s.step(1)
        sims.append(s)
    return sims


def assert_same(a_sims, b_sims, what):
    for k, (a, b) in enumerate(zip(a_sims, b_sims)):
        sa, sb = a.get_state(), b.get_state()
        if sa != sb:
            x = np.frombuffer(sa, np.uint8)
            y = np.frombuffer(sb, np.uint8)
            bad = np.flatnonzero(x != y)
            raise AssertionError(f"{what}: member {k} {SPECS[k] if k < len(SPECS) else ''} differs from its "
                                 f"single-lattice run at {bad.size} bytes (first at {bad[0]})")


def test_batch_matches_single_lattice_runs(gpu):
    print(f"  members {SPECS}", flush=True)
    A = make_members(SPECS)
    B = make_members(SPECS)
    batch = dsm.Batch(A)
    assert batch.items(2) > 0 and batch.items(3) > 0
    # odd, then even step counts
    batch.step(7)
    for s in B:
        s.step(7)
    assert_same(A, B, "7 steps")
    batch.step(4)
    for s in B:
        s.step(4)
    assert_same(A, B, "11 steps")
    # a member stepped on its own between batch calls (its parity flips)
    A[2].step(1)
    B[2].step(1)
    A[5].step(3)
    B[5].step(3)
    batch.step(3)
    for s in B:
        s.step(3)
    assert_same(A, B, "after single steps of two members")
    assert [s.steps for s in A] == [s.steps for s in B]
    batch.close()


def test_every_schedule_gives_identical_results(gpu):
    A = make_members(SPECS)
    B = make_members(SPECS)
    batch = dsm.Batch(A)
    for dim in (2, 3):
        for v in range(dsm.dsm_tiling_variants(dim)):
            for planes, per_cu in ((1, 0), (5, 1), (16, 0), (64, 2)):
                batch.set_schedule(dim, v, planes, per_cu)
                assert batch.schedule(dim) == {"variant": v, "planes": planes, "blocks_per_cu": per_cu}
                batch.step(1)
                for s in B:
                    s.step(1)
                assert_same(A, B, f"schedule dim {dim} variant {v} planes {planes} per_cu {per_cu}")
    batch.close()


def test_tuner_keeps_state_and_results(gpu):
    """The tuner picks schedules from its model of the members' shapes and
    issues no step: states are untouched, and later steps still match the
    single-lattice runs bit for bit."""
    A = make_members(SPECS)
    B = make_members(SPECS)
    batch = dsm.Batch(A)
    before = [s.get_state() for s in A]
    c2, c3 = batch.tune()
    print(f"  tuned: 2D {batch.schedule(2)} cost {c2:.1f}, 3D {batch.schedule(3)} cost {c3:.1f}", flush=True)
    assert c2 > 0.0 and c3 > 0.0
    assert [s.get_state() for s in A] == before
    assert [s.steps for s in A] == [s.steps for s in B]
    batch.step(5)
    for s in B:
        s.step(5)
    assert_same(A, B, "after tuning")
    batch.close()


def test_measured_tuner_times_candidates_and_keeps_results(gpu):
    """The measured tuner times every candidate schedule on the batch itself
    and installs the fastest; the steps it takes leave the members where the
    same number of single-lattice steps would."""
    A = make_members(SPECS)
    B = make_members(SPECS)
    batch = dsm.Batch(A)
    s0 = [s.steps for s in A]
    ms2, ms3 = batch.tune(reps=2)
    taken = [s.steps - k for s, k in zip(A, s0)]
    print(f"  measured: 2D {batch.schedule(2)} {ms2:.4f} ms, 3D {batch.schedule(3)} {ms3:.4f} ms; "
          f"{taken[0]} steps taken", flush=True)
    assert ms2 > 0.0 and ms3 > 0.0
    assert len(set(taken)) == 1 and taken[0] >= 3 * 6 * 3
    for s in B:
        s.step(taken[0])
    assert_same(A, B, "after measured tuning")
    batch.step(3)
    for s in B:
        s.step(3)
    assert_same(A, B, "stepping after measured tuning")
    batch.close()


def test_fp16_batch_matches_single_lattice_runs(gpu):
    A = make_members(SPECS, storage=dsm.DSM_STORAGE_FP16)
    B = make_members(SPECS, storage=dsm.DSM_STORAGE_FP16)
    batch = dsm.Batch(A)
    batch.step(9)
    for s in B:
        s.step(9)
    assert_same(A, B, "FP16, 9 steps")
    batch.close()


def test_batched_member_matches_oracle(gpu):
    """A sinusoidal-wall drop stepped in a batch against the FP64 oracle
    (the same bar as the single-lattice parity: C within 1e-5)."""
    specs = [(2, (100, 37)), (3, (33, 9, 12)), (2, (64, 32))]
    A = make_members(specs)
    kappa, grav, C1, C2 = member_inputs(0, *specs[0])
    orc = Oracle(2, specs[0][1], kappa, gravity=grav, threads=8)
    orc.set_solid_field(C1)
    orc.set_liquid(C2)
    orc.step(1)
    batch = dsm.Batch(A)
    batch.step(399)
    orc.step(399)
    fg, fo = A[0].fields(), orc.fields()
    err = float(np.abs(fg["C2"] - fo["C2"]).max())
    erru = float(np.abs(fg["u"] - fo["u"]).max())
    print(f"  C2 max abs err {err:.3e}, u {erru:.3e}", flush=True)
    assert err < 1e-5 and erru < 1e-6
    orc.close()
    batch.close()


def test_batch_reports_an_unstable_member(gpu):
    specs = [(2, (64, 16)), (2, (64, 32))]
    A = make_members(specs)
    A[1].set_gravity((50.0, 0.0, 0.0))
    batch = dsm.Batch(A)
    with pytest.raises(dsm.DsmError) as e:
        batch.step(2000)
    assert e.value.code == dsm.DSM_EUNSTABLE
    assert "member 1" in str(e.value)
    batch.close()


def test_batch_argument_errors(gpu):
    specs = [(2, (64, 32)), (3, (33, 9, 12))]
    A = make_members(specs)
    fresh = make_members([(2, (64, 32))], first_step=False)[0]
    h16 = make_members([(2, (64, 32))], storage=dsm.DSM_STORAGE_FP16)[0]
    lib = dsm.load()
    arr = dsm._handles([s.handle for s in A])
    assert lib.dsm_batch_required_bytes(arr, 0) == 0
    assert lib.dsm_batch_required_bytes(None, 2) == 0
    assert dsm.dsm_batch_required_bytes([A[0].handle, A[0].handle]) == 0
    assert dsm.dsm_batch_required_bytes([A[0].handle, h16.handle]) == 0
    need = dsm.dsm_batch_required_bytes([s.handle for s in A])
    assert need > 0
    import torch

    buf = torch.empty(need + 512, dtype=torch.uint8, device=gpu)
    base = (buf.data_ptr() + 255) // 256 * 256
    stream = torch.cuda.current_stream(gpu).cuda_stream
    out = ctypes.c_void_p()
    assert lib.dsm_batch_create(arr, 2, ctypes.c_void_p(base), need - 1, ctypes.c_void_p(stream),
                                ctypes.byref(out)) == dsm.DSM_ENOMEM
    assert lib.dsm_batch_create(arr, 2, ctypes.c_void_p(base + 8), need, ctypes.c_void_p(stream),
                                ctypes.byref(out)) == dsm.DSM_EINVAL
    with pytest.raises(dsm.DsmError) as e:
        dsm.Batch([A[0], fresh])
    assert e.value.code == dsm.DSM_ESTATE
    batch = dsm.Batch(A)
    with pytest.raises(dsm.DsmError):
        batch.set_schedule(2, 7, 16)
    with pytest.raises(dsm.DsmError):
        batch.set_schedule(3, 0, 0)
    with pytest.raises(dsm.DsmError):
        batch.set_schedule(4, 0, 16)
    with pytest.raises(dsm.DsmError):
        batch.step(-1)
    with pytest.raises(dsm.DsmError):
        batch.tune(reps=1001)
    with pytest.raises(dsm.DsmError):
        batch.tune(reps=-1)
    batch.step(0)
    batch.close()
