"""ctypes wrapper of the FP64 CPU oracle (libdsm_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark.  The GPU package never imports this module.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsm_oracle.so")

CONFINE_PURPOSE = 0
CONFINE_AS_TYPESET = 1
FORCE_POTENTIAL = 0
FORCE_AS_TYPESET = 1
SOLID_RESET = 1
SOLID_REMASK = 2
EUNSTABLE = -4  # a step met a non-finite C or u

_dp = ctypes.POINTER(ctypes.c_double)


class _Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("kappa", ctypes.c_double * 3), ("alpha", ctypes.c_double), ("tau", ctypes.c_double),
        ("mobility", ctypes.c_double), ("gravity", ctypes.c_double * 3),
        ("confine_reading", ctypes.c_int), ("threads", ctypes.c_int),
        ("rho_liquid", ctypes.c_double), ("rho_gas", ctypes.c_double), ("tau_gas", ctypes.c_double),
        ("force_reading", ctypes.c_int),
    ]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build_oracle  # noqa: WPS433 (build on first use in tests)
        build_oracle.build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.dsmo_create.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.dsmo_destroy.argtypes = [ctypes.c_void_p]
    lib.dsmo_destroy.restype = None
    lib.dsmo_num_directions.argtypes = [ctypes.c_void_p]
    lib.dsmo_init_solid.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.dsmo_set_solid_field.argtypes = [ctypes.c_void_p, _dp]
    lib.dsmo_set_liquid.argtypes = [ctypes.c_void_p, _dp]
    lib.dsmo_set_gravity.argtypes = [ctypes.c_void_p, _dp]
    lib.dsmo_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.dsmo_free_energy.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.dsmo_mass.argtypes = [ctypes.c_void_p, _dp]
    lib.dsmo_fields.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
    lib.dsmo_chemical_potential.argtypes = [ctypes.c_void_p, _dp]
    lib.dsmo_get_populations.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.dsmo_set_populations.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.dsmo_set_postcollision.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.dsmo_get_mask.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.dsmo_link_q.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_int]
    lib.dsmo_link_q.restype = ctypes.c_double
    lib.dsmo_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp]
    lib.dsmo_equilibrium_f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
    lib.dsmo_equilibrium_f.restype = None
    lib.dsmo_equilibrium_g.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
    lib.dsmo_equilibrium_g.restype = None
    lib.dsmo_forcing.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.dsmo_forcing.restype = None
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"oracle {what} failed with code {rc}")
        self.code = rc


def _check(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


def lattice(dim):
    lib = load()
    c = (ctypes.c_int * 57)()
    w = np.zeros(19)
    Q = lib.dsmo_lattice(dim, c, _ptr(w))
    return np.array(c[: 3 * Q]).reshape(Q, 3), w[:Q].copy()


def equilibrium_f(dim, p_tilde, rho, u):
    lib = load()
    out = np.zeros(19)
    lib.dsmo_equilibrium_f(dim, p_tilde, rho, _ptr(_f64(u)), _ptr(out))
    return out[: 9 if dim == 2 else 19].copy()


def equilibrium_g(dim, C, mu, u):
    lib = load()
    out = np.zeros(19)
    lib.dsmo_equilibrium_g(dim, C, mu, _ptr(_f64(u)), _ptr(out))
    return out[: 9 if dim == 2 else 19].copy()


def forcing(dim, tau, rho, u, grad_rho, F):
    lib = load()
    out = np.zeros(19)
    lib.dsmo_forcing(dim, tau, rho, _ptr(_f64(u)), _ptr(_f64(grad_rho)), _ptr(_f64(F)), _ptr(out))
    return out[: 9 if dim == 2 else 19].copy()


class Oracle:
    """FP64 reference simulation; method names follow the GPU library's calls."""

    def __init__(self, dim, shape, kappa, alpha=1.0, tau=1.0, mobility=0.1,
                 gravity=(0.0, 0.0, 0.0), mask=None, threads=1,
                 confine_reading=CONFINE_PURPOSE, rho=(1.0, 1.0), tau_gas=None,
                 force_reading=FORCE_POTENTIAL):
        """rho = (rho_2, rho_3) of liquid and gas; tau_gas = tau_3 (default:
        tau, i.e. no viscosity contrast); force_reading selects the form of
        the surface-tension force (FORCE_POTENTIAL: mu grad C, the form used
        throughout; FORCE_AS_TYPESET: -C grad mu)."""
        lib = load()
        nx, ny = shape[0], shape[1]
        nz = shape[2] if dim == 3 else 1
        self.dim, self.shape = dim, (nx, ny, nz)
        self.N = nx * ny * nz
        p = _Params()
        p.dim, p.nx, p.ny, p.nz = dim, nx, ny, nz
        p.kappa[:] = [float(k) for k in kappa]
        p.alpha, p.tau, p.mobility = float(alpha), float(tau), float(mobility)
        p.gravity[:] = [float(g) for g in gravity]
        p.confine_reading, p.threads = int(confine_reading), int(threads)
        p.rho_liquid, p.rho_gas = float(rho[0]), float(rho[1])
        p.tau_gas = float(tau if tau_gas is None else tau_gas)
        p.force_reading = int(force_reading)
        h = ctypes.c_void_p()
        m = None
        if mask is not None:
            self._mask = np.ascontiguousarray(np.asarray(mask).reshape(-1), dtype=np.uint8)
            m = self._mask.ctypes.data_as(ctypes.c_void_p)
        _check(lib.dsmo_create(ctypes.byref(p), m, ctypes.byref(h)), "create")
        self._h = h
        self.Q = lib.dsmo_num_directions(h)
        self._lib = lib

    def close(self):
        if self._h:
            self._lib.dsmo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- fields are flat arrays in node order x + nx*(y + ny*z)
    def init_solid(self, n_steps, beta, omega, tau_s=1.0, mobility_s=1.0 / 6.0, flags=SOLID_RESET):
        _check(self._lib.dsmo_init_solid(self._h, int(n_steps), beta, omega, tau_s, mobility_s, int(flags)),
               "init_solid")

    def set_solid_field(self, C1):
        a = _f64(np.asarray(C1).reshape(-1))
        _check(self._lib.dsmo_set_solid_field(self._h, _ptr(a)), "set_solid_field")

    def set_liquid(self, C2):
        a = _f64(np.asarray(C2).reshape(-1))
        _check(self._lib.dsmo_set_liquid(self._h, _ptr(a)), "set_liquid")

    def set_gravity(self, g):
        a = _f64(list(g) + [0.0] * (3 - len(g)))
        _check(self._lib.dsmo_set_gravity(self._h, _ptr(a)), "set_gravity")

    def step(self, n):
        _check(self._lib.dsmo_step(self._h, int(n)), "step")

    def free_energy(self):
        F, E = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.dsmo_free_energy(self._h, ctypes.byref(F), ctypes.byref(E)), "free_energy")
        return F.value, E.value

    def mass(self):
        m = np.zeros(3)
        _check(self._lib.dsmo_mass(self._h, _ptr(m)), "mass")
        return m

    def fields(self):
        N, d = self.N, self.dim
        C1, C2, C3, p = (np.zeros(N) for _ in range(4))
        u = np.zeros(d * N)
        _check(self._lib.dsmo_fields(self._h, _ptr(C1), _ptr(C2), _ptr(C3), _ptr(u), _ptr(p)), "fields")
        return {"C1": C1, "C2": C2, "C3": C3, "u": u.reshape(d, N), "p": p}

    def chemical_potential(self):
        mu = np.zeros(self.N)
        _check(self._lib.dsmo_chemical_potential(self._h, _ptr(mu)), "chemical_potential")
        return mu

    def get_populations(self):
        f = np.zeros((self.Q, self.N))
        g = np.zeros((self.Q, self.N))
        _check(self._lib.dsmo_get_populations(self._h, _ptr(f), _ptr(g)), "get_populations")
        return f, g

    def set_populations(self, f, g):
        f, g = _f64(f), _f64(g)
        _check(self._lib.dsmo_set_populations(self._h, _ptr(f), _ptr(g)), "set_populations")

    def set_postcollision(self, fs, gs):
        fs, gs = _f64(fs), _f64(gs)
        _check(self._lib.dsmo_set_postcollision(self._h, _ptr(fs), _ptr(gs)), "set_postcollision")

    def mask(self):
        m = np.zeros(self.N, dtype=np.uint8)
        _check(self._lib.dsmo_get_mask(self._h, m.ctypes.data_as(ctypes.c_void_p)), "get_mask")
        return m

    def link_q(self, node, k):
        return self._lib.dsmo_link_q(self._h, int(node), int(k))
