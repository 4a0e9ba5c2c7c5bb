"""Seeded synthetic inputs shared by the library tests, the oracle tests and
the benchmark.

This module holds only initial data and mesh descriptions: no graph
quantities, fluxes, wave speeds or limiter arithmetic.  Every generator is
deterministic in its arguments (NumPy ``default_rng`` / PCG64 for random
draws).  States are returned in structure-of-arrays layout ``U[c, i]`` with
``c = 0`` density, ``1..dim`` momentum, ``dim+1`` total energy, and nodes
numbered lexicographically with x fastest.

Mesh convention: ``n`` counts nodes per direction.  A periodic direction of
length L has mesh size L/n; a direction bounded by walls has (hi-lo)/(n-1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    dim: int
    n: tuple
    lo: tuple
    hi: tuple
    periodic: tuple

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    def spacing(self):
        return tuple((self.hi[d] - self.lo[d]) /
                     (self.n[d] if self.periodic[d] else self.n[d] - 1)
                     for d in range(self.dim))

    def coords(self):
        """Node coordinates, shape (dim, N), x fastest."""
        h = self.spacing()
        axes = [self.lo[d] + h[d] * np.arange(self.n[d]) for d in range(self.dim)]
        grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
        return np.stack([g.reshape(-1) for g in grids])


def conserved(rho, vel, p, gamma):
    """(rho, v, p) -> (rho, rho v, p/(gamma-1) + rho |v|^2 / 2)."""
    rho = np.asarray(rho, np.float64)
    vel = [np.asarray(v, np.float64) for v in vel]
    dim = len(vel)
    U = np.empty((dim + 2,) + rho.shape)
    U[0] = rho
    ke = np.zeros_like(rho)
    for k, v in enumerate(vel):
        U[1 + k] = rho * v
        ke += 0.5 * rho * v * v
    U[dim + 1] = p / (gamma - 1.0) + ke
    return U


# ---------------------------------------------------------------------------
# Isentropic vortex on the periodic square [-5, 5]^2 (strength beta).
# ---------------------------------------------------------------------------
def vortex_mesh(n: int) -> Mesh:
    return Mesh(2, (n, n), (-5.0, -5.0), (5.0, 5.0), (True, True))


def vortex_state(n: int, t: float = 0.0, beta: float = 5.0, gamma: float = 1.4,
                 u_inf=(1.0, 1.0)):
    """Exact isentropic vortex translated by u_inf * t; the vortex centre and
    its periodic images are taken at the nearest periodic offset."""
    mesh = vortex_mesh(n)
    x, y = mesh.coords()
    L = 10.0
    xc, yc = u_inf[0] * t, u_inf[1] * t
    dx = (x - xc + 0.5 * L) % L - 0.5 * L
    dy = (y - yc + 0.5 * L) % L - 0.5 * L
    r2 = dx * dx + dy * dy
    f = beta / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    u = u_inf[0] - f * dy
    v = u_inf[1] + f * dx
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi * np.pi) * \
        np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return mesh, conserved(rho, (u, v), p, gamma)


# ---------------------------------------------------------------------------
# Four-quadrant Riemann data on [0,1]^2 with reflecting walls.
# ---------------------------------------------------------------------------
def quadrant_states(seed: int):
    """Per quadrant (SW, SE, NW, NE): rho log-uniform in [0.1, 2],
    p uniform in [0.05, 1], u and v uniform in [-1, 1]; drawn in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = float(np.exp(rng.uniform(np.log(0.1), np.log(2.0))))
        p = float(rng.uniform(0.05, 1.0))
        u = float(rng.uniform(-1.0, 1.0))
        v = float(rng.uniform(-1.0, 1.0))
        out.append((rho, u, v, p))
    return out


def four_quadrant_mesh(n: int) -> Mesh:
    return Mesh(2, (n, n), (0.0, 0.0), (1.0, 1.0), (False, False))


def four_quadrant_state(n: int, seed: int = 0, gamma: float = 1.4):
    mesh = four_quadrant_mesh(n)
    x, y = mesh.coords()
    q = (x >= 0.5).astype(int) + 2 * (y >= 0.5).astype(int)
    st = np.array(quadrant_states(seed))
    rho, u, v, p = st[q, 0], st[q, 1], st[q, 2], st[q, 3]
    return mesh, conserved(rho, (u, v), p, gamma)


# ---------------------------------------------------------------------------
# 3D Mach-3 shock tube along x in [0,1]^3 with seeded 1% density noise.
# ---------------------------------------------------------------------------
def shock_tube_mesh(n: int) -> Mesh:
    return Mesh(3, (n, n, n), (0.0,) * 3, (1.0,) * 3, (False,) * 3)


def mach3_post_shock(gamma: float = 1.4, rho1: float = 1.4, p1: float = 1.0,
                     mach: float = 3.0):
    """Rankine-Hugoniot state behind a normal shock of Mach number `mach`
    moving into gas at rest (rho1, p1)."""
    a1 = np.sqrt(gamma * p1 / rho1)
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    u2 = mach * a1 * (1.0 - rho1 / rho2)
    return rho2, u2, p2


def shock_tube_state(n: int, seed: int = 0, gamma: float = 1.4,
                     x_shock: float = 0.25, noise: float = 0.01):
    mesh = shock_tube_mesh(n)
    x = mesh.coords()[0]
    rho2, u2, p2 = mach3_post_shock(gamma)
    post = x < x_shock
    rho = np.where(post, rho2, 1.4)
    u = np.where(post, u2, 0.0)
    p = np.where(post, p2, 1.0)
    rng = np.random.default_rng(seed)
    rho = rho * (1.0 + noise * rng.uniform(-1.0, 1.0, size=rho.shape))
    zero = np.zeros_like(rho)
    return mesh, conserved(rho, (u, zero, zero), p, gamma)


# ---------------------------------------------------------------------------
# 1D Riemann problems embedded in a y-periodic 2D strip.
# ---------------------------------------------------------------------------
RIEMANN_1D = {
    # name: (rho_L, u_L, p_L, rho_R, u_R, p_R, final time)
    "sod": (1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 0.2),
    "lax": (0.445, 0.698, 3.528, 0.5, 0.0, 0.571, 0.13),
    "toro2": (1.0, -2.0, 0.4, 1.0, 2.0, 0.4, 0.1),
}


def strip_mesh(nx: int, ny: int = 4) -> Mesh:
    return Mesh(2, (nx, ny), (0.0, 0.0), (1.0, ny / (nx - 1.0)), (False, True))


def riemann_strip_state(name: str, nx: int, ny: int = 4, gamma: float = 1.4,
                        x0: float = 0.5):
    rl, ul, pl, rr, ur, pr, _ = RIEMANN_1D[name]
    mesh = strip_mesh(nx, ny)
    x = mesh.coords()[0]
    left = x < x0
    rho = np.where(left, rl, rr)
    u = np.where(left, ul, ur)
    p = np.where(left, pl, pr)
    return mesh, conserved(rho, (u, np.zeros_like(u)), p, gamma)


def constant_state(mesh: Mesh, rho=1.0, vel=None, p=1.0, gamma=1.4):
    vel = vel if vel is not None else (0.0,) * mesh.dim
    ones = np.ones(mesh.N)
    return conserved(rho * ones, tuple(v * ones for v in vel), p * ones, gamma)


def random_smooth_state(mesh: Mesh, seed: int = 0, gamma: float = 1.4,
                        amp: float = 0.3):
    """Smooth seeded perturbation of a uniform state (for invariant tests)."""
    rng = np.random.default_rng(seed)
    X = mesh.coords()
    L = [mesh.hi[d] - mesh.lo[d] for d in range(mesh.dim)]
    def field():
        ph = rng.uniform(0, 2 * np.pi, size=mesh.dim)
        k = rng.integers(1, 3, size=mesh.dim)
        s = np.ones(mesh.N)
        for d in range(mesh.dim):
            s = s * np.sin(2 * np.pi * k[d] * (X[d] - mesh.lo[d]) / L[d] + ph[d])
        return s
    rho = 1.0 + amp * field()
    p = 1.0 + amp * field()
    vel = tuple(0.5 * amp * field() for _ in range(mesh.dim))
    return conserved(rho, vel, p, gamma)


def random_rough_state(mesh: Mesh, seed: int = 0, gamma: float = 1.4):
    """Node-wise independent seeded states (strong jumps everywhere)."""
    rng = np.random.default_rng(seed)
    rho = np.exp(rng.uniform(np.log(0.1), np.log(2.0), size=mesh.N))
    p = rng.uniform(0.05, 1.0, size=mesh.N)
    vel = tuple(rng.uniform(-1.0, 1.0, size=mesh.N) for _ in range(mesh.dim))
    return conserved(rho, vel, p, gamma)


# ---------------------------------------------------------------------------
# Serving: independent four-quadrant requests of different sizes.
# ---------------------------------------------------------------------------
def serving_requests(count: int = 256, seed: int = 0, nmin: int = 64,
                     nmax: int = 1024, rate: float = 20.0):
    """Request stream: arrival times of a Poisson process with `rate` per
    second, mesh sizes N x N with N log-uniform in [nmin, nmax] (rounded),
    and a data seed per request.  Returns a list of (t_arrival, n, seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    n = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=count))).astype(int)
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return [(float(t[k]), int(n[k]), int(seeds[k])) for k in range(count)]


def nr_vortex_state(n: int = 80, mach: float = 0.5, vbar: float = 0.75, r0: float = 0.25,
                    gamma: float = 1.4):
    """Vortex convected through [-1,1]^2 by a uniform stream (the
    non-reflecting boundary tests of the paper's Sec. 6.2): rho = 1,
    v = v_inf + vbar/r0 psi(|x|) (-y, x), p = p_inf - rho vbar^2 psi^2 / 2,
    psi(r) = exp((1 - r^2/r0^2)/2), v_inf = (1, 0), a_inf = 1/mach,
    p_inf = a_inf^2/gamma; centre 0 and r0 = 0.25 (not given in the paper).
    Returns (mesh, U, far-field state U_inf)."""
    mesh = Mesh(2, (n, n), (-1.0, -1.0), (1.0, 1.0), (False, False))
    x, y = mesh.coords()
    psi = np.exp(0.5 * (1.0 - (x * x + y * y) / r0 ** 2))
    p_inf = (1.0 / mach) ** 2 / gamma
    u = 1.0 - vbar / r0 * psi * y
    v = vbar / r0 * psi * x
    p = p_inf - 0.5 * vbar ** 2 * psi ** 2
    rho = np.ones_like(x)
    U = np.vstack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
    U_inf = np.array([1.0, 1.0, 0.0, p_inf / (gamma - 1.0) + 0.5])
    return mesh, U, U_inf
