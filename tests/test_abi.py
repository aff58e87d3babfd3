"""The C ABI without a GPU: libdsm.so loads, exports every function that
include/dsm.h declares, sizes its device buffer, and rejects invalid
arguments before it issues any device work."""
import ctypes
import os
import re

import pytest

from paper_2504_19941_amd import dsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(dsm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dsm.LIB_PATH):
        from paper_2504_19941_amd import build

        build.build()
    return dsm.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dsm_create", "dsm_step", "dsm_free_energy", "dsm_fields", "dsm_mass",
                     "dsm_init_solid", "dsm_set_liquid", "dsm_destroy", "dsm_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in include/dsm.h but not exported"
    assert sorted(dsm.EXPORTED) == sorted(declared_functions())


def good_params(**kw):
    p = dsm.make_params(3, (32, 24, 16), (0.01, 0.005, 0.01))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_required_bytes_matches_layout(lib):
    p = good_params()
    N = 32 * 24 * 16
    need = dsm.dsm_required_bytes(p)
    # four FP32 population sets of 19 planes dominate the buffer
    assert need >= 4 * 19 * N * 4 + N * 4 + N
    assert need < 4 * 19 * N * 4 + 24 * N * 4 + (1 << 20)
    p2 = dsm.make_params(2, (64, 32), (0.01, 0.005, 0.01))
    assert dsm.dsm_required_bytes(p2) >= 4 * 9 * 64 * 32 * 4


@pytest.mark.parametrize("field,value", [
    ("dim", 4), ("nx", 3), ("nz", 2), ("tau", 0.5), ("tau", float("nan")), ("mobility", 0.0),
    ("alpha", 0.0), ("reduce_every", -1), ("kernel", 7),
])
def test_invalid_params_rejected_on_host(lib, field, value):
    p = good_params(**{field: value})
    assert dsm.dsm_required_bytes(p) == 0
    h = ctypes.c_void_p()
    rc = lib.dsm_create(ctypes.byref(p), None, ctypes.c_void_p(256), ctypes.c_size_t(1 << 40), None,
                        ctypes.byref(h))
    assert rc == dsm.DSM_EINVAL
    assert h.value is None
    assert dsm.dsm_last_error() != ""


def test_negative_kappa_and_zero_fluid_kappa(lib):
    p = good_params()
    p.kappa[0] = -1.0
    assert dsm.dsm_required_bytes(p) == 0
    p = good_params()
    p.kappa[1] = p.kappa[2] = 0.0
    assert dsm.dsm_required_bytes(p) == 0


def test_small_or_misaligned_buffer_rejected(lib):
    p = good_params()
    need = dsm.dsm_required_bytes(p)
    h = ctypes.c_void_p()
    rc = lib.dsm_create(ctypes.byref(p), None, ctypes.c_void_p(4096), ctypes.c_size_t(need - 1), None,
                        ctypes.byref(h))
    assert rc == dsm.DSM_ENOMEM
    assert "too small" in dsm.dsm_last_error()
    rc = lib.dsm_create(ctypes.byref(p), None, ctypes.c_void_p(4096 + 8), ctypes.c_size_t(need), None,
                        ctypes.byref(h))
    assert rc == dsm.DSM_EINVAL
    rc = lib.dsm_create(ctypes.byref(p), None, None, ctypes.c_size_t(need), None, ctypes.byref(h))
    assert rc == dsm.DSM_EINVAL


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.dsm_step(None, 1) == dsm.DSM_EINVAL
    assert lib.dsm_destroy(None) == dsm.DSM_EINVAL
    assert lib.dsm_free_energy(None, None, None) == dsm.DSM_EINVAL
    assert lib.dsm_tiling_variants(3) >= 1
    assert lib.dsm_tiling_variants(5) == 0
    assert lib.dsm_get_tiling(None, None, None) == dsm.DSM_EINVAL


def test_storage_modes_size_the_buffer(lib):
    shape = (64, 24, 16)  # rows of 64 elements fill whole 128-byte lines in both storages
    p32 = dsm.make_params(3, shape, (0.01, 0.005, 0.01))
    p16 = dsm.make_params(3, shape, (0.01, 0.005, 0.01))
    p16.storage = dsm.DSM_STORAGE_FP16
    n32, n16 = dsm.dsm_required_bytes(p32), dsm.dsm_required_bytes(p16)
    N = 64 * 24 * 16
    # four population buffers of Q planes shrink from 4 to 2 bytes per element
    assert n32 - n16 >= 4 * 19 * N * 2 - 4 * 256
    assert dsm.dsm_required_bytes(good_params(storage=3)) == 0


@pytest.mark.parametrize("nx,storage,pitch", [(32, 0, 32), (33, 0, 64), (100, 0, 128), (127, 0, 128),
                                              (32, 1, 64), (65, 1, 128), (128, 1, 128)])
def test_population_rows_are_padded_to_whole_lines(lib, nx, storage, pitch):
    """Population and rest-plane rows take a pitch of whole 128-byte lines:
    the buffer grows by exactly the padding of the four population sets (Q
    elements per padded node) and the two FP64 rest planes."""
    ny, nz = 6, 5
    es = 2 if storage else 4
    p = dsm.make_params(3, (nx, ny, nz), (0.01, 0.005, 0.01))
    p.storage = storage
    q = dsm.make_params(3, (pitch, ny, nz), (0.01, 0.005, 0.01))
    q.storage = storage
    need, need_pitch = dsm.dsm_required_bytes(p), dsm.dsm_required_bytes(q)
    rows = ny * nz
    pad_nodes = (pitch - nx) * rows
    # node-indexed arrays (C1, mask, fields, link records) shrink with the
    # real node count; populations and rest planes keep the padded size
    per_node_dense = need_pitch - need
    pops = 4 * 19 * pitch * rows * es + 2 * 8 * pitch * rows
    assert need >= pops
    assert 0 <= per_node_dense <= pad_nodes * 400 + 16 * 256


def test_batch_calls_reject_invalid_arguments_without_a_device(lib):
    """Batch calls validate their arguments on the host: NULL or empty member
    lists, NULL handles and NULL outputs never reach the device."""
    vp = ctypes.c_void_p
    arr = (vp * 2)()
    assert lib.dsm_batch_required_bytes(None, 3) == 0
    assert lib.dsm_batch_required_bytes(arr, 0) == 0
    assert lib.dsm_batch_required_bytes(arr, 2) == 0  # NULL members
    out = vp()
    assert lib.dsm_batch_create(arr, 2, vp(1 << 20), 1 << 20, None, None) == dsm.DSM_EINVAL
    assert lib.dsm_batch_create(arr, 2, vp(1 << 20), 1 << 20, None, ctypes.byref(out)) == dsm.DSM_EINVAL
    assert out.value is None
    assert "NULL" in dsm.dsm_last_error()
    s = dsm.dsm_batch_schedule(0, 16, 0)
    assert lib.dsm_batch_set_schedule(None, 2, ctypes.byref(s)) == dsm.DSM_EINVAL
    assert lib.dsm_batch_get_schedule(None, 2, ctypes.byref(s)) == dsm.DSM_EINVAL
    assert lib.dsm_batch_tune(None, 2, None) == dsm.DSM_EINVAL
    assert lib.dsm_batch_step(None, 1) == dsm.DSM_EINVAL
    assert lib.dsm_batch_step_timed(None, 1, None) == dsm.DSM_EINVAL
    assert lib.dsm_batch_size(None) == -1
    assert lib.dsm_batch_items(None, 2) == -1
    assert lib.dsm_batch_destroy(None) == dsm.DSM_EINVAL


def test_size_limits_are_checked_on_host(lib):
    """The largest lattices: a plane of populations must stay below 2 GiB
    (32-bit buffer offsets within a plane) and the lattice below 2^32
    population slots; beyond either limit the size is 0 and dsm_create
    fails with DSM_EINVAL before touching the device."""
    # 3D plane: (nx + 64) * ny * 19 * 4 bytes
    ok = dsm.make_params(3, (4096, 6000, 4), (0.01, 0.005, 0.01))
    assert dsm.dsm_required_bytes(ok) > 0
    big_plane = dsm.make_params(3, (8192, 3500, 4), (0.01, 0.005, 0.01))
    assert dsm.dsm_required_bytes(big_plane) == 0
    h = ctypes.c_void_p()
    rc = lib.dsm_create(ctypes.byref(big_plane), None, ctypes.c_void_p(256), ctypes.c_size_t(1 << 50), None,
                        ctypes.byref(h))
    assert rc == dsm.DSM_EINVAL and "2 GiB" in dsm.dsm_last_error()
    # total slots: (nx + 64) * ny * nz * 19 > 2^32 - 1
    many = dsm.make_params(3, (1024, 1024, 256), (0.01, 0.005, 0.01))
    assert dsm.dsm_required_bytes(many) == 0
    rc = lib.dsm_create(ctypes.byref(many), None, ctypes.c_void_p(256), ctypes.c_size_t(1 << 50), None,
                        ctypes.byref(h))
    assert rc == dsm.DSM_EINVAL and "2^32" in dsm.dsm_last_error()
    # a 2D lattice of 2^28 nodes is fine (planes are single rows)
    assert dsm.dsm_required_bytes(dsm.make_params(2, (16384, 16384), (0.01, 0.005, 0.01))) > 0


def test_field_selection_is_checked_before_the_library_is_called():
    with pytest.raises(ValueError):
        dsm.dsm_fields(None, 16, 2, which=("C2", "rho"))
    with pytest.raises(ValueError):
        dsm.dsm_fields(None, 16, 2, which="rho")
