"""Second, independent FP64 oracle of the same step, in vectorised NumPy.

TEST INFRASTRUCTURE ONLY.  It is written separately from the C oracle
(whole-field array operations with periodic rolls instead of per-node loops;
its own lattice construction) so that agreement of the two to round-off pins
both against a transcription slip in either.  It is meant for small lattices
(16 x 16, 8^3).

It also offers plain halfway bounce-back (the population leaving towards
the wall returns reversed at the same node) as a textbook special case of
the interpolated rule: for a wall lying half-way between nodes the two must
coincide.

Readings are the same as the C oracle's (stated there): the surface-tension
force in the potential form mu grad C, the half-force velocity correction
with the total force, the rest population of g_eq closing the zeroth moment,
s_i with -u.u / (2 c_s^2), the confining potential acting on solid outside
and fluid inside S, the Omega terms acting outside [0, 1], and for the
density and viscosity contrast the floored fraction C2 / (C2 + C3) and the
step H(x) = 1 for x > 0.
"""
from __future__ import annotations

import itertools

import numpy as np

CS2 = 1.0 / 3.0


def lattice(dim):
    """Velocities and weights.  D2Q9 as listed in the paper; D3Q19 built
    from the speed classes {0, axis, face diagonal}, each velocity followed
    by its opposite, in the same order the libraries use."""
    if dim == 2:
        c = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, 1], [-1, -1], [1, -1], [-1, 1]])
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
        return c, w
    vel = [(0, 0, 0)]
    for a in range(3):
        e = [0, 0, 0]
        e[a] = 1
        vel += [tuple(e), tuple(-v for v in e)]
    for a, b in itertools.combinations(range(3), 2):
        for sb in (1, -1):
            e = [0, 0, 0]
            e[a], e[b] = 1, sb
            vel += [tuple(e), tuple(-v for v in e)]
    c = np.array(vel)
    w = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int((v ** 2).sum())] for v in c])
    return c, w


class MiniOracle:
    def __init__(self, dim, shape, kappa, alpha=1.0, tau=1.0, mobility=0.1, gravity=(0.0, 0.0, 0.0),
                 mask=None, bounce="interpolated", rho=(1.0, 1.0), tau_gas=None):
        self.dim, self.shape = dim, tuple(shape)
        self.rho2, self.rho3 = rho
        self.tau3 = tau if tau_gas is None else tau_gas
        self.c, self.w = lattice(dim)
        self.Q = len(self.w)
        self.k1, self.k2, self.k3 = kappa
        self.alpha, self.tau = alpha, tau
        self.tau_g = 0.5 + mobility / CS2
        self.grav = np.array(gravity[:dim], dtype=float)
        self.mask = np.zeros(self.shape, bool) if mask is None else np.asarray(mask).astype(bool)
        self.bounce = bounce
        self.C1 = self.mask.astype(float)
        self.stage = 0

    # -- stencils ---------------------------------------------------------
    def at(self, a, ci):
        """a(x + c_i) for every x."""
        return np.roll(a, shift=tuple(-int(v) for v in ci), axis=tuple(range(self.dim)))

    def from_(self, a, ci):
        """a(x - c_i) for every x."""
        return np.roll(a, shift=tuple(int(v) for v in ci), axis=tuple(range(self.dim)))

    def lap(self, a):
        return 2.0 / CS2 * sum(wi * (self.at(a, ci) - a) for ci, wi in zip(self.c, self.w))

    def grad(self, a):
        return np.stack([sum(wi * ci[d] * self.at(a, ci) for ci, wi in zip(self.c, self.w)) / CS2
                         for d in range(self.dim)])

    # -- set-up -------------------------------------------------------------
    def set_solid_field(self, C1):
        self.C1 = np.array(C1, dtype=float)

    def _mu(self, phi):
        a2 = self.alpha ** 2
        if self.stage == 2:
            S = self.C1 + phi
            return (self.k2 * phi * (1 - phi) * (1 - 2 * phi) + self.k3 * S * (1 - S) * (1 - 2 * S)
                    - a2 * self.k2 * self.lap(phi) - a2 * self.k3 * (self.lap(self.C1) + self.lap(phi)))
        k13 = self.k1 + self.k3
        active = ((phi < 0.5) & self.mask) | ((phi > 0.5) & ~self.mask)
        m = k13 * phi * (1 - phi) * (1 - 2 * phi) - a2 * k13 * self.lap(phi)
        m = m + np.where(active, 2 * self.beta * (phi - 0.5), 0.0)
        m = m + np.where(phi < 0, 2 * self.omega * phi, 0.0) - np.where(phi > 1, 2 * self.omega * (1 - phi), 0.0)
        return m

    def _geq(self, C, mu, u):
        out = np.empty((self.Q,) + self.shape)
        for i in range(1, self.Q):
            out[i] = self.w[i] * (mu + C * self._s(i, u))
        out[0] = C - out[1:].sum(axis=0)
        return out

    def _s(self, i, u):
        cu = np.tensordot(self.c[i].astype(float), u, axes=1)
        uu = (u ** 2).sum(axis=0)
        return cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2)

    def _init(self, phi):
        self.f = np.zeros((self.Q,) + self.shape)
        self.g = self._geq(phi, self._mu(phi), np.zeros((self.dim,) + self.shape))

    def set_liquid(self, C2):
        self.stage = 2
        self._init(np.array(C2, dtype=float))

    def init_solid(self, n_steps, beta, omega, tau_s=1.0, mobility_s=1.0 / 6.0, reset=True, remask=False):
        self.beta, self.omega = beta, omega
        self._tau_s, self._tau_gs = tau_s, 0.5 + mobility_s / CS2
        if reset or self.stage != 1:
            self.stage = 1
            self._init(self.mask.astype(float))
        for _ in range(n_steps):
            self._step()
        self.C1 = self.g.sum(axis=0)
        if remask:
            self.mask = self.C1 > 0.5

    def set_postcollision(self, fs, gs):
        """State = streaming of the given post-collision arrays [Q][N] (node
        order x fastest)."""
        if self.stage == 0:
            self.stage = 2
        self._stream(self._unflat(fs), self._unflat(gs))

    def _unflat(self, a):
        a = np.asarray(a, dtype=float).reshape(self.Q, -1)
        return np.stack([row.reshape(self.shape, order="F") for row in a])

    # -- one step -------------------------------------------------------------
    def _solid(self):
        return (self.C1 > 0.5) if self.stage == 2 else np.zeros(self.shape, bool)

    def observe(self):
        phi = self.g.sum(axis=0)
        mu = self._mu(phi)
        solid = self._solid()
        F = mu * self.grad(phi)
        if self.stage == 2:
            F = F + phi * self.grav.reshape((self.dim,) + (1,) * self.dim)
        F[:, solid] = 0.0
        rho = self._density(phi)
        grho = self.grad(rho)
        mom = np.tensordot(self.c.T.astype(float), self.f, axes=1)
        u = (mom + 0.5 * F) / rho
        u[:, solid] = 0.0
        p = self.f.sum(axis=0) + 0.5 * (u * grho).sum(axis=0)
        p[solid] = 0.0
        self._rho, self._grho = rho, grho
        return phi, mu, F, u, p, solid

    def _density(self, phi):
        """rho_3 + (rho_2 - rho_3) C2 / (C2 + C3), the fraction's denominator
        1 - C1 floored at 1e-6 and the fraction clipped to [0, 1]; 1 in the
        solid stage."""
        if self.stage != 2:
            return np.ones(self.shape)
        frac = np.clip(phi / np.maximum(1.0 - self.C1, 1e-6), 0.0, 1.0)
        return self.rho3 + (self.rho2 - self.rho3) * frac

    def _step(self):
        phi, mu, F, u, p, solid = self.observe()
        rho, grho = self._rho, self._grho
        if self.stage == 1:
            tau = np.full(self.shape, self._tau_s)
        else:
            C3 = 1.0 - self.C1 - phi
            tau = np.where(phi - C3 > 0.0, self.tau, self.tau3)
        tau_g = self._tau_gs if self.stage == 1 else self.tau_g
        fs = np.empty_like(self.f)
        for i in range(self.Q):
            ci = self.c[i].astype(float)
            s = self._s(i, u)
            feq = self.w[i] * (p + rho * s)
            cu_grad = np.tensordot(ci, grho, axes=1) - (u * grho).sum(axis=0)
            Fi = (1 - 0.5 / tau) * self.w[i] * (cu_grad * s + np.tensordot(ci, F, axes=1) / CS2)
            fs[i] = self.f[i] - (self.f[i] - feq) / tau + Fi
        fs[:, solid] = 0.0
        geq = self._geq(phi, mu, u)
        gs = self.g - (self.g - geq) / tau_g
        self._stream(fs, gs)

    def _stream(self, fs, gs):
        solid = self._solid()
        self.g = np.stack([self.from_(gs[i], self.c[i]) for i in range(self.Q)])
        f = np.stack([self.from_(fs[i], self.c[i]) for i in range(self.Q)])
        opp = [0] + [i + 1 if i % 2 else i - 1 for i in range(1, self.Q)]
        if solid.any():
            G = self.grad(self.C1)
            gn = np.sqrt((G ** 2).sum(axis=0))
            xi = 2 * self.alpha * np.arctanh(np.clip(1 - 2 * self.C1, 0.0, 1 - 1e-12))
            for i in range(1, self.Q):
                cut = ~solid & self.from_(solid, self.c[i])
                if not cut.any():
                    continue
                k = opp[i]
                if self.bounce == "halfway":
                    f[i] = np.where(cut, fs[k], f[i])
                    continue
                ck = self.c[k].astype(float)
                ln = np.sqrt((ck ** 2).sum())
                with np.errstate(divide="ignore", invalid="ignore"):
                    cosnc = np.tensordot(ck, G, axes=1) / (gn * ln)
                    q = np.clip(xi / cosnc / ln, 0.0, 1.0)
                q = np.where((gn < 1e-12) | ~(cosnc > 1e-6), 0.5, q)
                down_solid = self.at(solid, self.c[i])
                near = (q < 0.5) & ~down_solid
                qq = np.where(down_solid & (q < 0.5), 0.5, q)
                v_near = 2 * q * fs[k] + (1 - 2 * q) * self.at(fs[k], self.c[i])
                with np.errstate(divide="ignore", invalid="ignore"):
                    v_far = fs[k] / (2 * qq) + (2 * qq - 1) / (2 * qq) * fs[i]
                f[i] = np.where(cut, np.where(near, v_near, v_far), f[i])
        f[:, solid] = 0.0
        self.f = f

    def step(self, n):
        for _ in range(n):
            self._step()

    # -- outputs in node order (x fastest) ------------------------------------
    def _flat(self, a):
        return np.asarray(a).reshape(-1, order="F")

    def fields(self):
        phi, mu, F, u, p, solid = self.observe()
        C1 = self.C1 if self.stage == 2 else phi
        C2 = phi if self.stage == 2 else np.zeros(self.shape)
        return {"C1": self._flat(C1), "C2": self._flat(C2), "C3": self._flat(1 - C1 - C2),
                "u": np.stack([self._flat(u[d]) for d in range(self.dim)]), "p": self._flat(CS2 * p),
                "mu": self._flat(mu)}

    def populations(self):
        return (np.stack([self._flat(a) for a in self.f]), np.stack([self._flat(a) for a in self.g]))
