"""Seeded synthetic inputs shaped like the paper's lattice Boltzmann workloads.

This module holds geometry and initial-condition generators only: solid
masks, analytic diffuse-solid fields, liquid drops and slabs, the interfacial
parameters of a target contact angle, and seeded random population states for
parity checks.  It holds none of the step's arithmetic and is shared by the
tests, the benchmark and the oracle-side checks.

Arrays are returned with shape (nx, ny) or (nx, ny, nz) and must be flattened
in Fortran order (x fastest) to match the libraries' node order
n = x + nx*(y + ny*z); :func:`flat` does that.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def flat(a: np.ndarray) -> np.ndarray:
    """Flatten an (nx, ny[, nz]) array to node order n = x + nx*(y + ny*z)."""
    return np.ascontiguousarray(np.asarray(a).reshape(-1, order="F"))


def unflat(v: np.ndarray, shape) -> np.ndarray:
    """Inverse of :func:`flat`."""
    return np.asarray(v).reshape(shape, order="F")


# ---------------------------------------------------------------------------
# interfacial parameters

def kappas_from_tensions(g12: float, g13: float, g23: float, alpha: float = 1.0):
    """kappa_1..3 from the three pairwise tensions (Sec. II.A: inversion of
    gamma_nm = alpha (kappa_n + kappa_m) / 6)."""
    k1 = 3.0 / alpha * (g12 + g13 - g23)
    k2 = 3.0 / alpha * (g12 - g13 + g23)
    k3 = 3.0 / alpha * (-g12 + g13 + g23)
    return (k1, k2, k3)


def kappas_for_angle(theta_deg: float, gamma: float = 2.5e-3, alpha: float = 1.0):
    """kappa_1..3 for a target equilibrium angle, with the liquid-gas and
    solid-liquid tensions both fixed at ``gamma`` and the solid-gas tension
    set by Young's law (the convention of Supp. D)."""
    g12 = g23 = gamma
    g13 = g12 + g23 * math.cos(math.radians(theta_deg))
    return kappas_from_tensions(g12, g13, g23, alpha)


# ---------------------------------------------------------------------------
# geometry helpers

def tanh_profile(d: np.ndarray, alpha: float = 1.0) -> np.ndarray:
    """1/2 + 1/2 tanh(d / (2 alpha)) of a signed distance d (positive inside)."""
    return 0.5 + 0.5 * np.tanh(np.asarray(d, dtype=np.float64) / (2.0 * alpha))


def _coords(shape):
    return np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")


def periodic_slab_distance(coord: np.ndarray, lo: float, hi: float, period: int) -> np.ndarray:
    """Signed distance (positive inside) to the periodic slab lo <= s <= hi."""
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    r = np.abs(((coord - mid + 0.5 * period) % period) - 0.5 * period)
    return half - r


def min_image(d: np.ndarray, period: int) -> np.ndarray:
    return (d + 0.5 * period) % period - 0.5 * period


def drop_field(shape, center, radius, C1=None, alpha: float = 1.0,
               open_axis: int | None = None) -> np.ndarray:
    """Liquid drop: tanh-smoothed disc / ball of ``radius`` at ``center``,
    cut to the fluid side by (1 - C1).  Distances use the minimum image
    except along ``open_axis`` (the wall normal of a sessile drop), where the
    plain difference is used so that the drop does not wrap through the wall
    into the far side of the box."""
    X = _coords(shape)
    r2 = np.zeros(shape)
    for d, (xd, c) in enumerate(zip(X, center)):
        dd = xd - c if d == open_axis else min_image(xd - c, shape[d])
        r2 += dd ** 2
    C2 = tanh_profile(radius - np.sqrt(r2), alpha)
    if C1 is not None:
        C2 = C2 * (1.0 - C1)
    return C2


@dataclass
class Workload:
    """One lattice problem: geometry, parameters and initial liquid."""
    name: str
    dim: int
    shape: tuple
    kappa: tuple
    alpha: float = 1.0
    tau: float = 1.0
    mobility: float = 0.1
    gravity: tuple = (0.0, 0.0, 0.0)
    mask: np.ndarray | None = None      # solid region S (uint8)
    C1: np.ndarray | None = None        # diffuse solid (analytic), or None -> solid stage
    C2: np.ndarray | None = None        # initial liquid
    wall_level: float | None = None     # C1 = 1/2 plane of a flat wall (for angle fits)
    wall_axis: int = 1
    solid_stage: dict = field(default_factory=dict)
    seed: int = 0
    rho: tuple = (1.0, 1.0)             # densities of liquid and gas
    tau_gas: float | None = None        # relaxation time of the gas (None: tau)

    @property
    def nodes(self) -> int:
        return int(np.prod(self.shape))


def flat_wall(dim: int, shape, thickness: int, alpha: float = 1.0):
    """Solid slab occupying the first ``thickness`` layers along the last
    axis; its C1 is the analytic tanh of the periodic signed distance, with
    the faces half-way between nodes."""
    axis = dim - 1
    X = _coords(shape)
    lo, hi = -0.5, thickness - 0.5
    d = periodic_slab_distance(X[axis], lo, hi, shape[axis])
    mask = (d > 0).astype(np.uint8)
    return mask, tanh_profile(d, alpha), hi


def sessile_drop(dim: int, shape, thickness: int, radius: float, theta_deg: float,
                 seed: int = 0, noise: float = 0.0, alpha: float = 1.0,
                 tau: float = 1.0, mobility: float = 0.1, name: str = "sessile") -> Workload:
    """Drop (semicircle / hemisphere) centred on a flat diffuse wall."""
    mask, C1, face = flat_wall(dim, shape, thickness, alpha)
    center = [0.5 * n for n in shape]
    center[dim - 1] = face
    C2 = drop_field(shape, center, radius, C1, alpha, open_axis=dim - 1)
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        C2 = C2 + noise * rng.uniform(-1.0, 1.0, size=shape) * (C1 < 0.5)
    return Workload(name=name, dim=dim, shape=tuple(shape), kappa=kappas_for_angle(theta_deg),
                    alpha=alpha, tau=tau, mobility=mobility, mask=mask, C1=C1, C2=C2,
                    wall_level=face, wall_axis=dim - 1, seed=seed)


def config_2d_contact_angle(theta_deg: float, seed: int = 1, noise: float = 0.0) -> Workload:
    """D2Q9 128x64 periodic, 8-node bottom wall, semicircular drop R = 25."""
    return sessile_drop(2, (128, 64), 8, 25.0, theta_deg, seed=seed, noise=noise,
                        name=f"d2q9-128x64-wall8-R25-theta{theta_deg:g}")


def config_3d_sessile(theta_deg: float, n: int = 128, seed: int = 2, noise: float = 0.0,
                      radius: float = 30.0, thickness: int = 6) -> Workload:
    """D3Q19 n^3 periodic, 6-node bottom slab, hemispherical drop R = 30."""
    return sessile_drop(3, (n, n, n), thickness, radius, theta_deg, seed=seed, noise=noise,
                        name=f"d3q19-{n}^3-slab{thickness}-R{radius:g}-theta{theta_deg:g}")


def pillar_mask(shape, base: int = 8, width: int = 8, pitch: int = 16, height: int = 32,
                jitter: int = 2, seed: int = 3) -> np.ndarray:
    """Square micropillars on a base slab (z < base), pillars of ``width``
    on a ``pitch`` lattice, each offset by a seeded integer jitter."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    mask = np.zeros(shape, dtype=np.uint8)
    mask[:, :, :base] = 1
    for px in range(nx // pitch):
        for py in range(ny // pitch):
            jx, jy = rng.integers(-jitter, jitter + 1, size=2)
            x0 = px * pitch + (pitch - width) // 2 + int(jx)
            y0 = py * pitch + (pitch - width) // 2 + int(jy)
            xs = np.arange(x0, x0 + width) % nx
            ys = np.arange(y0, y0 + width) % ny
            mask[np.ix_(xs, ys, np.arange(base, base + height))] = 1
    return mask


def config_3d_pillars(shape=(256, 256, 192), theta_deg: float = 120.0, seed: int = 3,
                      liquid=(44, 104)) -> Workload:
    """Micropillar array with a liquid slab above it; C1 comes from the solid
    stage (5000 steps, beta = 1e-3, Omega = 2e-4)."""
    mask = pillar_mask(shape, seed=seed)
    X = _coords(shape)
    C2 = tanh_profile(periodic_slab_distance(X[2], liquid[0], liquid[1], shape[2]))
    return Workload(name=f"d3q19-{shape[0]}x{shape[1]}x{shape[2]}-pillars", dim=3,
                    shape=tuple(shape), kappa=kappas_for_angle(theta_deg), mask=mask, C1=None,
                    C2=C2, gravity=(0.0, 0.0, -1e-5),
                    solid_stage=dict(n_steps=5000, beta=1e-3, omega=2e-4), seed=seed)


def pillar_field(shape, base: int = 8, width: int = 8, pitch: int = 16, height: int = 32,
                 jitter: int = 2, seed: int = 3, alpha: float = 1.0) -> np.ndarray:
    """Analytic diffuse solid of the micropillar array of :func:`pillar_mask`
    (same seed, same jitter draws): C1 = tanh profile of the signed distance
    to the union of the base slab and the square pillars (box distances,
    faces half-way between nodes, positive inside).  Each pillar is evaluated
    on a window around it; pillars are at least 4 nodes apart."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    Z = np.arange(nz, dtype=np.float64)
    d = np.broadcast_to(periodic_slab_distance(Z, -0.5, base - 0.5, nz), shape).copy()
    m = 6  # window margin (the tanh profile is flat beyond a few nodes)
    zlo, zhi = base - 0.5, base + height - 0.5
    zw = np.arange(max(0, base - m), min(nz, base + height + m))
    for px in range(nx // pitch):
        for py in range(ny // pitch):
            jx, jy = rng.integers(-jitter, jitter + 1, size=2)
            x0 = px * pitch + (pitch - width) // 2 + int(jx)
            y0 = py * pitch + (pitch - width) // 2 + int(jy)
            xs = np.arange(x0 - m, x0 + width + m)
            ys = np.arange(y0 - m, y0 + width + m)
            X, Y, Zc = np.meshgrid(xs.astype(float), ys.astype(float), zw.astype(float), indexing="ij")
            lo = np.array([x0 - 0.5, y0 - 0.5, zlo])
            hi = np.array([x0 + width - 0.5, y0 + width - 0.5, zhi])
            P = np.stack([X, Y, Zc])
            below, above = lo.reshape(3, 1, 1, 1) - P, P - hi.reshape(3, 1, 1, 1)
            outside = np.sqrt((np.maximum(np.maximum(below, above), 0.0) ** 2).sum(axis=0))
            inside = np.minimum(-below, -above).min(axis=0)
            sd = np.where(outside > 0.0, -outside, inside)
            win = np.ix_(xs % nx, ys % ny, zw)
            d[win] = np.maximum(d[win], sd)
    return tanh_profile(d, alpha)


def config_3d_pillars_analytic(shape=(256, 256, 192), theta_deg: float = 120.0, seed: int = 3,
                               liquid=(44, 104)) -> Workload:
    """The micropillar workload with the analytic diffuse solid of
    :func:`pillar_field` in place of the solid stage (parity tests give both
    sides this same C1)."""
    w = config_3d_pillars(shape, theta_deg, seed, liquid)
    w.C1 = pillar_field(shape, seed=seed)
    w.C2 = w.C2 * (1.0 - w.C1)
    w.name += "-analytic-C1"
    return w


def sinusoid_mask(shape, amplitude: float, wavelength: float, base: float) -> np.ndarray:
    """2D solid below y_s(x) = base + A sin(2 pi x / lambda)."""
    X, Y = _coords(shape)
    ys = base + amplitude * np.sin(2.0 * np.pi * X / wavelength)
    return (Y <= ys).astype(np.uint8)


def sinusoid_surface(shape, amplitude: float, wavelength: float, base: float, alpha: float = 1.0):
    """2D diffuse solid below y_s(x) = base + A sin(2 pi x / lambda): C1 is
    the tanh profile of the signed distance to the surface, taken to first
    order as (y_s(x) - y) / sqrt(1 + y_s'(x)^2); the mask is C1 > 1/2."""
    X, Y = _coords(shape)
    k = 2.0 * np.pi / wavelength
    ys = base + amplitude * np.sin(k * X)
    slope = amplitude * k * np.cos(k * X)
    d = (ys - Y) / np.sqrt(1.0 + slope ** 2)
    C1 = tanh_profile(d, alpha)
    return (C1 > 0.5).astype(np.uint8), C1


BATCH_2D_RECIPE = ("(nx 64-512, ny 32-256; sinusoidal walls A 2-12, lambda 16-128; drops R 15-40; "
                   "theta 45-135 deg; body force 1e-7-1e-5)")


def batch_2d_sinusoid(count: int = 512, seed: int = 4, size_lo=(64, 32), size_hi=(512, 256)) -> list:
    """Independent D2Q9 drops on sinusoidally undulated walls, all drawn from
    one seed: lattice nx in [64, 512] and ny in [32, 256] (uniform integers),
    amplitude 2-12 nodes, wavelength 16-128 rounded so that a whole number of
    periods fits the periodic x extent, drop radius 15-40 clipped to what the
    lattice holds, contact angle 45-135 degrees, body force 1e-7-1e-5
    (log-uniform) along x.  The wall's troughs sit 4 nodes above the bottom."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(rng.integers(size_lo[0], size_hi[0] + 1))
        ny = int(rng.integers(size_lo[1], size_hi[1] + 1))
        amp = float(rng.uniform(2.0, 12.0))
        lam = float(rng.uniform(16.0, 128.0))
        lam = nx / max(1, round(nx / lam))
        base = amp + 4.0
        radius = float(rng.uniform(15.0, 40.0))
        radius = max(4.0, min(radius, 0.4 * nx, ny - base - amp - 4.0))
        theta = float(rng.uniform(45.0, 135.0))
        g = float(10.0 ** rng.uniform(-7.0, -5.0))
        shape = (nx, ny)
        mask, C1 = sinusoid_surface(shape, amp, lam, base)
        xc = 0.5 * nx
        yc = base + amp * np.sin(2.0 * np.pi * xc / lam)
        C2 = drop_field(shape, (xc, yc), radius, C1, open_axis=1)
        out.append(Workload(name=f"d2q9-{nx}x{ny}-sin{amp:.1f}x{lam:.1f}-R{radius:.1f}-theta{theta:.0f}",
                            dim=2, shape=shape, kappa=kappas_for_angle(theta), mask=mask, C1=C1, C2=C2,
                            gravity=(g, 0.0, 0.0), seed=seed * 100003 + k))
    return out


def capillary_channel(width: int, length: int, theta_deg: float, gravity: float, wall: int = 4,
                      alpha: float = 1.0, seed: int = 0, tau: float = 1.0, tau_gas: float = 0.52) -> Workload:
    """D3Q19 capillary filling: a square duct of ``width`` nodes (walls
    ``wall`` thick on each side, so the periodic box is width + 2 wall
    across) along x, fed from a liquid reservoir.  The duct axis is the
    lattice's fastest axis, so a long duct fills whole wavefronts.  An end
    plate fills x < wall; the reservoir x in [wall, xr) has no side walls,
    the duct starts at xr = length / 4, and the liquid fills the reservoir up
    to xr + 2.  Gravity -g along x.  C1 is the tanh profile of the signed
    distance to the solid (union of duct walls and end plate, each a max/min
    of plane distances).  The default relaxation times give the kinematic
    viscosities 1/6 (liquid) and 2/300 (gas) of the paper's capillary-filling
    runs, at equal densities."""
    n = width + 2 * wall
    shape = (length, n, n)
    X, Y, Z = _coords(shape)
    c = 0.5 * (n - 1)
    xr = length // 4
    d_side = np.maximum(np.abs(Y - c), np.abs(Z - c)) - 0.5 * width        # > 0 inside the side walls
    d_duct = np.minimum(d_side, X - (xr - 0.5))                              # walls only for x >= xr
    d_plate = periodic_slab_distance(X, -0.5, wall - 0.5, length)
    C1 = tanh_profile(np.maximum(d_duct, d_plate), alpha)
    liquid = tanh_profile(np.minimum(X - (wall - 0.5), (xr + 2.0) - X), alpha)
    C2 = liquid * (1.0 - C1)
    return Workload(name=f"d3q19-channel-w{width}-L{length}-theta{theta_deg:.0f}", dim=3, shape=shape,
                    kappa=kappas_for_angle(theta_deg), alpha=alpha, mask=(C1 > 0.5).astype(np.uint8),
                    C1=C1, C2=C2, gravity=(-gravity, 0.0, 0.0), seed=seed, tau=tau, tau_gas=tau_gas)


def particle_at_interface(n: int, radius: float, theta_deg: float, alpha: float = 1.0,
                          seed: int = 0) -> Workload:
    """D3Q19 n^3 periodic box with a diffuse spherical particle centred on
    a flat liquid-gas interface: liquid fills n/8 <= z < n/2, the particle
    centre sits on z = n/2 (the centre is offset by a seeded sub-node
    shift)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    X, Y, Z = _coords(shape)
    ctr = 0.5 * n + rng.uniform(-0.5, 0.5, size=3)
    r = np.sqrt(sum(min_image(Xd - cd, n) ** 2 for Xd, cd in zip((X, Y, Z), ctr)))
    C1 = tanh_profile(radius - r, alpha)
    C2 = tanh_profile(periodic_slab_distance(Z, n / 8.0, ctr[2], n), alpha) * (1.0 - C1)
    return Workload(name=f"d3q19-particle-{n}^3-R{radius:.1f}-theta{theta_deg:.0f}", dim=3, shape=shape,
                    kappa=kappas_for_angle(theta_deg), alpha=alpha, mask=(C1 > 0.5).astype(np.uint8),
                    C1=C1, C2=C2, seed=seed)


SERVE_RECIPE = ("Poisson arrivals; half capillary-filling jobs (square duct width 8-32, length 128-512, "
                "gravity 1e-6-1e-5, theta 30-80 deg, liquid/gas viscosity 1/6 vs 2/300), half "
                "particle-at-interface jobs (n^3 box n 96-160, particle radius 10-20, theta 45-135 deg)")


def serve_jobs(count: int, seed: int = 5, steps=(200, 1000), small: bool = False) -> list:
    """The job mix of the served form, drawn from one seed: (workload, steps)
    pairs, alternating at random between the two kinds.  ``small`` shrinks
    every lattice (for tests) while keeping both kinds."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        if rng.uniform() < 0.5:
            width = int(rng.integers(8, 33))
            length = int(rng.integers(128, 513))
            if small:
                width, length = max(6, width // 4), max(24, length // 8)
            g = float(10.0 ** rng.uniform(-6.0, -5.0))
            w = capillary_channel(width, length, float(rng.uniform(30.0, 80.0)), g, seed=seed * 7919 + k)
        else:
            n = int(rng.integers(96, 161))
            radius = float(rng.uniform(10.0, 20.0))
            if small:
                n, radius = max(24, n // 4), max(4.0, radius / 4)
            w = particle_at_interface(n, radius, float(rng.uniform(45.0, 135.0)), seed=seed * 7919 + k)
        # fields held in node order (x fastest), as a client hands them to the
        # library, so that flat() is a view
        w.C1, w.C2 = np.asfortranarray(w.C1), np.asfortranarray(w.C2)
        if w.mask is not None:
            w.mask = np.asfortranarray(w.mask)
        out.append((w, int(rng.integers(steps[0], steps[1] + 1))))
    return out


def random_postcollision_state(Q: int, shape, C2: np.ndarray, seed: int, amp: float = 1e-3):
    """Seeded random post-collision populations around a liquid field:
    f* = amp * U(-1, 1); g*_0 = C2 + amp * U(-1, 1); g*_i = amp * U(-1, 1)
    for i > 0 (index 0 is the rest direction in both libraries)."""
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    fs = amp * rng.uniform(-1.0, 1.0, size=(Q, N))
    gs = amp * rng.uniform(-1.0, 1.0, size=(Q, N))
    gs[0] += flat(C2)
    return fs, gs
