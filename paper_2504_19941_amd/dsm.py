"""Python binding of libdsm.so (include/dsm.h): argument marshalling only.

Every function named ``dsm_*`` here calls the C function of the same name;
all lattice work runs in the library's HIP kernels.  PyTorch supplies the
device buffer and the stream, nothing else.  If libdsm.so has not been built
this module raises on first use: there is no fallback implementation.

:class:`Simulation` bundles a handle with its device buffer.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdsm.so")

DSM_OK, DSM_EINVAL, DSM_ENOMEM, DSM_EDEVICE, DSM_EUNSTABLE, DSM_ESTATE = 0, -1, -2, -3, -4, -5
DSM_SOLID_RESET, DSM_SOLID_REMASK = 1, 2
DSM_KERNEL_FUSED, DSM_KERNEL_SPLIT = 0, 1
DSM_STORAGE_FP32, DSM_STORAGE_FP16 = 0, 1

EXPORTED = [
    "dsm_required_bytes", "dsm_create", "dsm_init_solid", "dsm_set_solid_field", "dsm_set_liquid",
    "dsm_set_gravity", "dsm_step", "dsm_step_timed", "dsm_free_energy", "dsm_mass", "dsm_diagnostics",
    "dsm_diagnostics_noalloc", "dsm_solid_region", "dsm_fields", "dsm_chemical_potential", "dsm_get_populations", "dsm_set_populations", "dsm_set_postcollision",
    "dsm_state_bytes", "dsm_get_state", "dsm_set_state", "dsm_step_count", "dsm_set_tiling",
    "dsm_get_tiling", "dsm_tiling_variants", "dsm_tune_tiling", "dsm_destroy", "dsm_last_error",
    "dsm_batch_required_bytes", "dsm_batch_create", "dsm_batch_set_schedule", "dsm_batch_get_schedule",
    "dsm_batch_tune", "dsm_batch_step", "dsm_batch_step_timed", "dsm_batch_size", "dsm_batch_items",
    "dsm_batch_destroy",
]

_dp = ctypes.POINTER(ctypes.c_double)


class dsm_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("kappa", ctypes.c_double * 3), ("alpha", ctypes.c_double), ("tau", ctypes.c_double),
        ("mobility", ctypes.c_double), ("gravity", ctypes.c_double * 3),
        ("reduce_every", ctypes.c_int), ("kernel", ctypes.c_int), ("storage", ctypes.c_int),
        ("rho", ctypes.c_double * 2), ("tau_gas", ctypes.c_double),
    ]


class dsm_batch_schedule(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("planes", ctypes.c_int), ("blocks_per_cu", ctypes.c_int)]


class dsm_diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double * 3), ("free_energy", ctypes.c_double),
                ("kinetic_energy", ctypes.c_double), ("max_speed", ctypes.c_double),
                ("nonfinite_nodes", ctypes.c_double)]


class DsmError(RuntimeError):
    def __init__(self, code, what, msg):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Loads libdsm.so and declares its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdsm.so not found at {path}: build it with "
                           "`python -m paper_2504_19941_amd.build` (no fallback exists)")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # the one that owns the device buffers and streams handed to it
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.dsm_required_bytes.argtypes = [ctypes.POINTER(dsm_params)]
    lib.dsm_required_bytes.restype = ctypes.c_size_t
    lib.dsm_create.argtypes = [ctypes.POINTER(dsm_params), vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.dsm_init_solid.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int]
    lib.dsm_set_solid_field.argtypes = [vp, _dp]
    lib.dsm_set_liquid.argtypes = [vp, _dp]
    lib.dsm_set_gravity.argtypes = [vp, _dp]
    lib.dsm_step.argtypes = [vp, ctypes.c_int]
    lib.dsm_step_timed.argtypes = [vp, ctypes.c_int, _dp, _dp]
    lib.dsm_free_energy.argtypes = [vp, _dp, _dp]
    lib.dsm_mass.argtypes = [vp, _dp]
    lib.dsm_diagnostics.argtypes = [vp, ctypes.POINTER(dsm_diag)]
    lib.dsm_diagnostics_noalloc.argtypes = [vp, ctypes.POINTER(dsm_diag)]
    lib.dsm_solid_region.argtypes = [vp, vp]
    lib.dsm_fields.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
    lib.dsm_chemical_potential.argtypes = [vp, _dp]
    lib.dsm_get_populations.argtypes = [vp, _dp, _dp]
    lib.dsm_set_populations.argtypes = [vp, _dp, _dp]
    lib.dsm_set_postcollision.argtypes = [vp, _dp, _dp]
    lib.dsm_state_bytes.argtypes = [vp]
    lib.dsm_state_bytes.restype = ctypes.c_size_t
    lib.dsm_get_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.dsm_set_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.dsm_step_count.argtypes = [vp]
    lib.dsm_step_count.restype = ctypes.c_longlong
    lib.dsm_set_tiling.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.dsm_get_tiling.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.dsm_tiling_variants.argtypes = [ctypes.c_int]
    lib.dsm_tune_tiling.argtypes = [vp, ctypes.c_int, _dp]
    lib.dsm_destroy.argtypes = [vp]
    lib.dsm_last_error.argtypes = []
    lib.dsm_last_error.restype = ctypes.c_char_p
    vpp = ctypes.POINTER(vp)
    sp = ctypes.POINTER(dsm_batch_schedule)
    lib.dsm_batch_required_bytes.argtypes = [vpp, ctypes.c_int]
    lib.dsm_batch_required_bytes.restype = ctypes.c_size_t
    lib.dsm_batch_create.argtypes = [vpp, ctypes.c_int, vp, ctypes.c_size_t, vp, vpp]
    lib.dsm_batch_set_schedule.argtypes = [vp, ctypes.c_int, sp]
    lib.dsm_batch_get_schedule.argtypes = [vp, ctypes.c_int, sp]
    lib.dsm_batch_tune.argtypes = [vp, ctypes.c_int, _dp]
    lib.dsm_batch_step.argtypes = [vp, ctypes.c_int]
    lib.dsm_batch_step_timed.argtypes = [vp, ctypes.c_int, _dp]
    lib.dsm_batch_size.argtypes = [vp]
    lib.dsm_batch_items.argtypes = [vp, ctypes.c_int]
    lib.dsm_batch_destroy.argtypes = [vp]
    _lib = lib
    return lib


def _check(rc, what):
    if rc != DSM_OK:
        raise DsmError(rc, what, dsm_last_error())


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


# ---------------------------------------------------------------------------
# one function per C entry point

def make_params(dim, shape, kappa, alpha=1.0, tau=1.0, mobility=0.1, gravity=(0.0, 0.0, 0.0),
                reduce_every=0, kernel=DSM_KERNEL_FUSED, storage=DSM_STORAGE_FP32, rho=(1.0, 1.0),
                tau_gas=0.0) -> dsm_params:
    p = dsm_params()
    p.dim = int(dim)
    p.nx, p.ny = int(shape[0]), int(shape[1])
    p.nz = int(shape[2]) if dim == 3 else 1
    p.kappa[:] = [float(k) for k in kappa]
    p.alpha, p.tau, p.mobility = float(alpha), float(tau), float(mobility)
    g = list(gravity) + [0.0] * (3 - len(gravity))
    p.gravity[:] = [float(v) for v in g]
    p.reduce_every, p.kernel, p.storage = int(reduce_every), int(kernel), int(storage)
    p.rho[:] = [float(rho[0]), float(rho[1])]
    p.tau_gas = float(tau_gas or 0.0)
    return p


def dsm_required_bytes(params: dsm_params) -> int:
    return int(load().dsm_required_bytes(ctypes.byref(params)))


def dsm_create(params: dsm_params, mask, dev_ptr: int, dev_bytes: int, stream: int):
    m = None
    if mask is not None:
        m = np.ascontiguousarray(np.asarray(mask).reshape(-1), dtype=np.uint8)
    h = ctypes.c_void_p()
    rc = load().dsm_create(ctypes.byref(params), None if m is None else m.ctypes.data_as(ctypes.c_void_p),
                           ctypes.c_void_p(dev_ptr), ctypes.c_size_t(dev_bytes), ctypes.c_void_p(stream),
                           ctypes.byref(h))
    _check(rc, "dsm_create")
    return h


def dsm_init_solid(h, n_steps, beta, omega, tau_s=1.0, mobility_s=1.0 / 6.0, flags=DSM_SOLID_RESET):
    _check(load().dsm_init_solid(h, int(n_steps), float(beta), float(omega), float(tau_s), float(mobility_s),
                                 int(flags)), "dsm_init_solid")


def dsm_set_solid_field(h, C1):
    a = _f64(C1)
    _check(load().dsm_set_solid_field(h, _p(a)), "dsm_set_solid_field")


def dsm_set_liquid(h, C2):
    a = _f64(C2)
    _check(load().dsm_set_liquid(h, _p(a)), "dsm_set_liquid")


def dsm_set_gravity(h, g):
    a = _f64(list(g) + [0.0] * (3 - len(g)))
    _check(load().dsm_set_gravity(h, _p(a)), "dsm_set_gravity")


def dsm_step(h, n):
    _check(load().dsm_step(h, int(n)), "dsm_step")


def dsm_step_timed(h, n):
    """n steps; returns (mean fused-kernel ms, mean link-kernel ms)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(load().dsm_step_timed(h, int(n), ctypes.byref(a), ctypes.byref(b)), "dsm_step_timed")
    return a.value, b.value


def dsm_free_energy(h):
    F, E = ctypes.c_double(), ctypes.c_double()
    _check(load().dsm_free_energy(h, ctypes.byref(F), ctypes.byref(E)), "dsm_free_energy")
    return F.value, E.value


def dsm_mass(h):
    m = np.zeros(3)
    _check(load().dsm_mass(h, _p(m)), "dsm_mass")
    return m


def _diag_dict(d):
    return {"mass": np.array(d.mass[:]), "free_energy": d.free_energy, "kinetic_energy": d.kinetic_energy,
            "max_speed": d.max_speed, "nonfinite_nodes": d.nonfinite_nodes}


def dsm_diagnostics(h):
    d = dsm_diag()
    _check(load().dsm_diagnostics(h, ctypes.byref(d)), "dsm_diagnostics")
    return _diag_dict(d)


def dsm_diagnostics_noalloc(h):
    d = dsm_diag()
    _check(load().dsm_diagnostics_noalloc(h, ctypes.byref(d)), "dsm_diagnostics_noalloc")
    return _diag_dict(d)


def dsm_solid_region(h, N):
    m = np.zeros(N, dtype=np.uint8)
    _check(load().dsm_solid_region(h, m.ctypes.data_as(ctypes.c_void_p)), "dsm_solid_region")
    return m


FIELDS = ("C1", "C2", "C3", "u", "p")


def dsm_fields(h, N, dim, which=FIELDS):
    """The requested fields (names from FIELDS, or one name) as FP64 host
    arrays; the library computes and copies only those."""
    if isinstance(which, str):
        which = (which,)
    bad = set(which) - set(FIELDS)
    if bad:
        raise ValueError(f"unknown fields {sorted(bad)}")
    out = {k: np.zeros(dim * N if k == "u" else N) for k in FIELDS if k in which}
    ptr = [_p(out[k]) if k in out else None for k in FIELDS]
    _check(load().dsm_fields(h, *ptr), "dsm_fields")
    if "u" in out:
        out["u"] = out["u"].reshape(dim, N)
    return out


def dsm_chemical_potential(h, N):
    mu = np.zeros(N)
    _check(load().dsm_chemical_potential(h, _p(mu)), "dsm_chemical_potential")
    return mu


def dsm_get_populations(h, Q, N):
    f = np.zeros((Q, N))
    g = np.zeros((Q, N))
    _check(load().dsm_get_populations(h, _p(f), _p(g)), "dsm_get_populations")
    return f, g


def dsm_set_populations(h, f, g):
    f, g = _f64(f), _f64(g)
    _check(load().dsm_set_populations(h, _p(f), _p(g)), "dsm_set_populations")


def dsm_set_postcollision(h, fs, gs):
    fs, gs = _f64(fs), _f64(gs)
    _check(load().dsm_set_postcollision(h, _p(fs), _p(gs)), "dsm_set_postcollision")


def dsm_state_bytes(h) -> int:
    return int(load().dsm_state_bytes(h))


def dsm_get_state(h) -> bytes:
    n = dsm_state_bytes(h)
    buf = ctypes.create_string_buffer(n)
    _check(load().dsm_get_state(h, buf, n), "dsm_get_state")
    return buf.raw


def dsm_set_state(h, state: bytes):
    buf = ctypes.create_string_buffer(state, len(state))
    _check(load().dsm_set_state(h, buf, len(state)), "dsm_set_state")


def dsm_step_count(h) -> int:
    return int(load().dsm_step_count(h))


def dsm_set_tiling(h, variant, planes):
    _check(load().dsm_set_tiling(h, int(variant), int(planes)), "dsm_set_tiling")


def dsm_get_tiling(h):
    v, p = ctypes.c_int(0), ctypes.c_int(0)
    _check(load().dsm_get_tiling(h, ctypes.byref(v), ctypes.byref(p)), "dsm_get_tiling")
    return v.value, p.value


def dsm_tune_tiling(h, reps=3) -> float:
    """Times every tile variant and march on the lattice itself (it advances
    by 1 + reps steps per candidate), installs the fastest; returns the fused
    kernel's ms per step under it."""
    ms = ctypes.c_double(0.0)
    _check(load().dsm_tune_tiling(h, int(reps), ctypes.byref(ms)), "dsm_tune_tiling")
    return ms.value


def dsm_tiling_variants(dim) -> int:
    return int(load().dsm_tiling_variants(int(dim)))


def dsm_destroy(h):
    _check(load().dsm_destroy(h), "dsm_destroy")


def dsm_last_error() -> str:
    return load().dsm_last_error().decode()


def _handles(handles):
    arr = (ctypes.c_void_p * len(handles))()
    for k, h in enumerate(handles):
        arr[k] = h.value if isinstance(h, ctypes.c_void_p) else h
    return arr


def dsm_batch_required_bytes(handles) -> int:
    return int(load().dsm_batch_required_bytes(_handles(handles), len(handles)))


def dsm_batch_create(handles, dev_ptr: int, dev_bytes: int, stream: int):
    h = ctypes.c_void_p()
    rc = load().dsm_batch_create(_handles(handles), len(handles), ctypes.c_void_p(dev_ptr),
                                 ctypes.c_size_t(dev_bytes), ctypes.c_void_p(stream), ctypes.byref(h))
    _check(rc, "dsm_batch_create")
    return h


def dsm_batch_set_schedule(b, dim, variant, planes, blocks_per_cu=0):
    s = dsm_batch_schedule(int(variant), int(planes), int(blocks_per_cu))
    _check(load().dsm_batch_set_schedule(b, int(dim), ctypes.byref(s)), "dsm_batch_set_schedule")


def dsm_batch_get_schedule(b, dim):
    s = dsm_batch_schedule()
    _check(load().dsm_batch_get_schedule(b, int(dim), ctypes.byref(s)), "dsm_batch_get_schedule")
    return {"variant": s.variant, "planes": s.planes, "blocks_per_cu": s.blocks_per_cu}


def dsm_batch_tune(b, reps=0):
    """reps == 0: installs the modelled best schedules and returns their
    modelled costs (2D, 3D) in wave-plane units.  reps > 0: times every
    candidate schedule on the batch itself (the members advance by the steps
    it takes), installs the fastest and returns its ms per step."""
    t = np.zeros(2)
    _check(load().dsm_batch_tune(b, int(reps), _p(t)), "dsm_batch_tune")
    return float(t[0]), float(t[1])


def dsm_batch_step(b, n):
    _check(load().dsm_batch_step(b, int(n)), "dsm_batch_step")


def dsm_batch_step_timed(b, n) -> float:
    ms = ctypes.c_double()
    _check(load().dsm_batch_step_timed(b, int(n), ctypes.byref(ms)), "dsm_batch_step_timed")
    return ms.value


def dsm_batch_size(b) -> int:
    return int(load().dsm_batch_size(b))


def dsm_batch_items(b, dim) -> int:
    return int(load().dsm_batch_items(b, int(dim)))


def dsm_batch_destroy(b):
    _check(load().dsm_batch_destroy(b), "dsm_batch_destroy")


# ---------------------------------------------------------------------------

class Simulation:
    """A libdsm.so handle together with the torch device buffer it lives in."""

    def __init__(self, dim, shape, kappa, alpha=1.0, tau=1.0, mobility=0.1, gravity=(0.0, 0.0, 0.0),
                 mask=None, reduce_every=0, kernel=DSM_KERNEL_FUSED, storage=DSM_STORAGE_FP32, device="cuda:0",
                 stream=None, dev_ptr=None, rho=(1.0, 1.0), tau_gas=0.0):
        """dev_ptr: optional 256-byte aligned device address of at least
        dsm_required_bytes bytes that the caller owns (e.g. a block of a
        larger arena); by default a torch buffer is allocated."""
        import torch

        self.dim = dim
        self.shape = tuple(shape)
        self.params = make_params(dim, shape, kappa, alpha, tau, mobility, gravity, reduce_every, kernel, storage,
                                  rho, tau_gas)
        self.N = int(self.params.nx * self.params.ny * self.params.nz)
        self.Q = 9 if dim == 2 else 19
        self.nbytes = dsm_required_bytes(self.params)
        if self.nbytes == 0:
            raise DsmError(DSM_EINVAL, "dsm_required_bytes", "invalid parameters")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if dev_ptr is None:
            # over-allocate by 256 bytes so the handle's base can be 256-byte aligned
            self.buffer = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
            self.base = (self.buffer.data_ptr() + 255) // 256 * 256
        else:
            self.buffer = None
            self.base = int(dev_ptr)
        self.handle = dsm_create(self.params, mask, self.base, self.nbytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            dsm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_solid(self, n_steps, beta, omega, tau_s=1.0, mobility_s=1.0 / 6.0, flags=DSM_SOLID_RESET):
        dsm_init_solid(self.handle, n_steps, beta, omega, tau_s, mobility_s, flags)

    def set_solid_field(self, C1):
        dsm_set_solid_field(self.handle, C1)

    def set_liquid(self, C2):
        dsm_set_liquid(self.handle, C2)

    def set_gravity(self, g):
        dsm_set_gravity(self.handle, g)

    def step(self, n):
        dsm_step(self.handle, n)

    def step_timed(self, n):
        return dsm_step_timed(self.handle, n)

    def free_energy(self):
        return dsm_free_energy(self.handle)

    def mass(self):
        return dsm_mass(self.handle)

    def fields(self, which=FIELDS):
        return dsm_fields(self.handle, self.N, self.dim, which)

    def diagnostics(self):
        return dsm_diagnostics(self.handle)

    def solid_region(self):
        return dsm_solid_region(self.handle, self.N)

    def chemical_potential(self):
        return dsm_chemical_potential(self.handle, self.N)

    def get_populations(self):
        return dsm_get_populations(self.handle, self.Q, self.N)

    def set_populations(self, f, g):
        dsm_set_populations(self.handle, f, g)

    def set_postcollision(self, fs, gs):
        dsm_set_postcollision(self.handle, fs, gs)

    def get_state(self) -> bytes:
        return dsm_get_state(self.handle)

    def set_state(self, state: bytes):
        dsm_set_state(self.handle, state)

    def set_tiling(self, variant, planes):
        dsm_set_tiling(self.handle, variant, planes)

    def tiling(self):
        """(variant, planes) of the fused step's launch shape in use."""
        return dsm_get_tiling(self.handle)

    def tune_tiling(self, reps=3):
        """Measured tiling tuner (dsm_tune_tiling): returns (variant, planes, ms)."""
        ms = dsm_tune_tiling(self.handle, reps)
        return (*self.tiling(), ms)

    @property
    def steps(self) -> int:
        return dsm_step_count(self.handle)


class Batch:
    """A libdsm.so batch over Simulation objects, with its torch device buffer.

    The Simulations must stay alive while the batch exists."""

    def __init__(self, sims, device="cuda:0", stream=None, dev_ptr=None):
        """dev_ptr: optional caller-owned 256-byte aligned device address of
        at least dsm_batch_required_bytes bytes (default: a torch buffer)."""
        import torch

        self.sims = list(sims)
        handles = [s.handle for s in self.sims]
        self.nbytes = dsm_batch_required_bytes(handles)
        if self.nbytes == 0:
            raise DsmError(DSM_EINVAL, "dsm_batch_required_bytes", "invalid members")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if dev_ptr is None:
            self.buffer = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
            base = (self.buffer.data_ptr() + 255) // 256 * 256
        else:
            self.buffer = None
            base = int(dev_ptr)
        self.handle = dsm_batch_create(handles, base, self.nbytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            dsm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedule(self, dim, variant, planes, blocks_per_cu=0):
        dsm_batch_set_schedule(self.handle, dim, variant, planes, blocks_per_cu)

    def schedule(self, dim):
        return dsm_batch_get_schedule(self.handle, dim)

    def tune(self, reps=0):
        return dsm_batch_tune(self.handle, reps)

    def step(self, n):
        dsm_batch_step(self.handle, n)

    def step_timed(self, n):
        return dsm_batch_step_timed(self.handle, n)

    def items(self, dim):
        return dsm_batch_items(self.handle, dim)

    @property
    def nodes(self) -> int:
        return sum(s.N for s in self.sims)
