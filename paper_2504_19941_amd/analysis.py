"""Host-side analysis of simulated fields: contact angle of a sessile drop.

The angle is measured as in Sec. III and IV of the paper: points on the
liquid-gas interface are fitted by a circle (a sphere in 3D) and the angle is
read where that circle meets the solid plane.  Details the paper leaves open:
  * the interface is the C2 = C3 level set, located by linear interpolation
    along every lattice line that crosses it;
  * points with C1 >= 0.01 or closer than 3 alpha to the wall plane are
    dropped, which removes the distortion near the contact line;
  * the fit is the algebraic (Kasa) least-squares circle/sphere;
  * cos(theta) = (wall_level - centre) / R along the wall normal.
The same function is applied to every field source, so it is analysis and
not part of the step.
"""
from __future__ import annotations

import math

import numpy as np


def interface_points(C1: np.ndarray, C2: np.ndarray, wall_axis: int, wall_level: float,
                     alpha: float = 1.0, c1_max: float = 0.01, clearance: float = 3.0):
    """Crossings of C2 = C3 along lattice lines, as an (n, dim) array."""
    C1 = np.asarray(C1, dtype=np.float64)
    C2 = np.asarray(C2, dtype=np.float64)
    phi = C2 - (1.0 - C1 - C2)
    dim = phi.ndim
    pts = []
    for ax in range(dim):
        a = phi
        b = np.roll(phi, -1, axis=ax)
        c1a = C1
        c1b = np.roll(C1, -1, axis=ax)
        cross = (a * b < 0.0)
        # do not connect across the periodic seam
        sl = [slice(None)] * dim
        sl[ax] = -1
        cross[tuple(sl)] = False
        idx = np.nonzero(cross)
        if len(idx[0]) == 0:
            continue
        fa, fb = a[idx], b[idx]
        t = fa / (fa - fb)
        c1 = c1a[idx] * (1.0 - t) + c1b[idx] * t
        coords = np.stack([i.astype(np.float64) for i in idx], axis=1)
        coords[:, ax] += t
        keep = (c1 < c1_max) & (coords[:, wall_axis] > wall_level + clearance * alpha)
        pts.append(coords[keep])
    if not pts:
        return np.zeros((0, dim))
    return np.concatenate(pts, axis=0)


def fit_circle(points: np.ndarray):
    """Algebraic least-squares circle / sphere: returns (centre, radius)."""
    P = np.asarray(points, dtype=np.float64)
    n, dim = P.shape
    if n < dim + 1:
        raise ValueError("not enough interface points for a fit")
    A = np.concatenate([P, np.ones((n, 1))], axis=1)
    b = -(P ** 2).sum(axis=1)
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    centre = -0.5 * sol[:dim]
    r2 = (centre ** 2).sum() - sol[dim]
    return centre, math.sqrt(max(r2, 0.0))


def contact_angle(C1: np.ndarray, C2: np.ndarray, wall_axis: int, wall_level: float,
                  alpha: float = 1.0) -> float:
    """Equilibrium contact angle (degrees) of a drop on a flat wall whose
    C1 = 1/2 plane lies at ``wall_level`` along ``wall_axis``."""
    pts = interface_points(C1, C2, wall_axis, wall_level, alpha)
    centre, R = fit_circle(pts)
    c = (wall_level - centre[wall_axis]) / R
    c = min(1.0, max(-1.0, c))
    return math.degrees(math.acos(c))
