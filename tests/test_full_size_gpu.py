"""GPU parity at the full workload sizes, in the configuration bench.py
times: 2D four-quadrant data on 4096x4096 nodes and the 3D Mach-3 shock tube
on 256^3 nodes, FP64, gamma = 1.4, c_cfl = 0.5, two limiter passes.

The oracle cannot run these meshes whole inside a test, so:
- the time step is checked against the oracle's value for the whole mesh,
  stored by tests/golden/make_full_size.py (1e-14 relative);
- one and two SSPRK(3,3) steps with that time step are checked on sampled
  blocks (corners, walls, the discontinuities, seeded interior points)
  against the oracle run on windows around them (tests/windows.py; the
  window method is itself checked against whole-mesh runs in
  test_oracle_window.py), to 1e-12 relative to the field's max norm;
- properties that hold at any size are checked on the whole result:
  admissibility, and conservation of mass and total energy with slip walls
  (global conservation lemma of Sec. 4).
"""
import json
import os

import numpy as np
import pytest

from paper_2106_02159_amd import abi, workloads as W
from tests.helpers import state_rel_err, state_scale
from tests.windows import oracle_window_step

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "full_size_dt.json")))
TOL = 1e-12


def say(*a):
    print(*a, flush=True)


def lumped_mass(mesh):
    """m_i of Q1 on a uniform box with walls: prod over directions of h
    (h/2 at the two end nodes)."""
    m = np.ones(1)
    for d in range(mesh.dim):
        h = mesh.spacing()[d]
        w = np.full(mesh.n[d], h)
        w[0] = w[-1] = 0.5 * h
        m = np.multiply.outer(w, m).reshape(-1)  # x fastest
    return m


def blocks(mesh, fixed, n_random, width, seed):
    rng = np.random.default_rng(seed)
    out = list(fixed)
    for _ in range(n_random):
        out.append(tuple(int(rng.integers(0, mesh.n[d] - width))
                         for d in range(mesh.dim)))
    return out


SETUPS = {
    # 2D: x = 0.5 lies between nodes 2047 and 2048; corners, walls, the
    # centre where all four quadrants meet, the interfaces, random interior
    "2d": dict(make=lambda: W.four_quadrant_state(4096, seed=0), width=16,
               fixed=[(0, 0), (4080, 4080), (0, 4080), (2040, 0), (0, 2040),
                      (2040, 2040), (2040, 900), (3100, 2040)],
               n_random=12, two_step=[(2040, 2040), (4080, 0), (0, 2040),
                                       (1234, 3210)]),
    # 3D: the shock starts at x = 0.25 (node 64); corners, edges, faces
    "3d": dict(make=lambda: W.shock_tube_state(256, seed=0), width=8,
               fixed=[(0, 0, 0), (248, 248, 248), (60, 0, 0), (60, 124, 124),
                      (60, 0, 124), (120, 248, 60)],
               n_random=4, two_step=[(62, 0, 127), (60, 124, 124)]),
}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("key", ["2d", "3d"])
def test_full_size(key):
    cfg = SETUPS[key]
    gold = GOLD[key]
    mesh, U0 = cfg["make"]()
    say("full size", key, mesh.n, "build")
    g = abi.Graph(mesh)
    s = abi.Solver(g, gamma=gold["gamma"], cfl=gold["cfl"])
    s.set_state(U0)  # projects the wall momentum, as bench.py does
    tau = gold["tau"]
    t_gpu = s.compute_dt()
    say("dt gpu", t_gpu, "oracle", tau)
    assert t_gpu == pytest.approx(tau, rel=1e-14, abs=0)
    Uin = s.get_state()
    say("step 1")
    s.step(tau)
    U1 = s.get_state()
    say("step 2")
    s.step(tau)
    U2 = s.get_state()
    del s

    # whole-field properties
    m = lumped_mass(mesh)
    for U in (U1, U2):
        dim = mesh.dim
        assert np.all(U[0] > 0)
        eps = U[dim + 1] - 0.5 * (U[1:1 + dim] ** 2).sum(axis=0) / U[0]
        assert np.all(eps > 0)
        for c in (0, dim + 1):
            a, b = np.dot(m, Uin[c]), np.dot(m, U[c])
            assert abs(b - a) <= 1e-12 * abs(a), (c, a, b)

    # sampled blocks against the oracle on windows
    scale = state_scale(U0)
    w = cfg["width"]
    for b in blocks(mesh, cfg["fixed"], cfg["n_random"], w, seed=7):
        say("window", b)
        idx, ref = oracle_window_step(mesh, U0, b, (w,) * mesh.dim, tau)
        err = state_rel_err(U1[:, idx], ref, scale=scale)
        say("  err", err.max())
        assert err.max() <= TOL, (key, b, err)
    wb = 4 if key == "3d" else 16
    for b in cfg["two_step"]:
        say("window, two steps", b)
        idx, ref = oracle_window_step(mesh, U0, b, (wb,) * mesh.dim, tau, steps=2)
        err = state_rel_err(U2[:, idx], ref, scale=scale)
        say("  err", err.max())
        assert err.max() <= TOL, (key, b, err)


@pytest.mark.timeout(900)
def test_full_size_navier_stokes_3d():
    """The Navier-Stokes configuration at 256^3: hyperbolic step tau,
    parabolic step 2 tau (mu = 1e-4, kappa = 1.4e-4, cv = 2.5, CG rtol
    1e-10), hyperbolic step tau -- the Strang step as separate calls, so
    that the parabolic step's properties can be checked on its own input:
    density unchanged bit for bit, wall velocity zero, total energy changed
    by exactly the kinetic energy removed at the no-slip nodes (to the CG
    tolerance), admissibility; mass conserved over the whole step."""
    gold = GOLD["3d"]
    mesh, U0 = W.shock_tube_state(256, seed=0)
    say("full size NS 3d build")
    g = abi.Graph(mesh)
    s = abi.Solver(g, gamma=gold["gamma"], cfl=gold["cfl"])
    s.set_state(U0)
    s.set_viscous(mu=1e-4, lam=0.0, kappa=1.4e-4, cv=2.5, cg_rtol=1e-10)
    tau = gold["tau"]
    Uin = s.get_state()
    s.step(tau)
    U1 = s.get_state()
    say("parabolic")
    s.step_parabolic(2.0 * tau)
    info = s.parabolic_info()
    say("  CG iterations", info.it_v, info.it_e, info.it_l, "fct", info.fct)
    assert 0 < info.it_v < 500 and 0 < info.it_e < 500
    U2 = s.get_state()
    s.step(tau)
    U3 = s.get_state()
    del s
    m = lumped_mass(mesh)
    assert np.array_equal(U2[0], U1[0])
    idx = np.indices(mesh.n[::-1]).reshape(3, -1)[::-1]
    wall = np.zeros(mesh.N, bool)
    for d in range(3):
        wall |= (idx[d] == 0) | (idx[d] == mesh.n[d] - 1)
    assert np.all(U2[1:4, wall] == 0.0)
    ke_wall = 0.5 * np.sum((m * np.sum(U1[1:4] ** 2, axis=0) / U1[0])[wall])
    dE = np.dot(m, U2[4]) - np.dot(m, U1[4])
    say("  energy change", dE, "wall kinetic energy", ke_wall)
    assert dE == pytest.approx(-ke_wall, abs=1e-9 * np.dot(m, U1[4]))
    for U in (U2, U3):
        eps = U[4] - 0.5 * (U[1:4] ** 2).sum(axis=0) / U[0]
        assert np.all(U[0] > 0) and np.all(eps > 0)
    a, b = np.dot(m, Uin[0]), np.dot(m, U3[0])
    assert abs(b - a) <= 1e-12 * a


def active_blocks(U_prev, U_next, dim, n, width, count, taken=()):
    """Block corners around the nodes whose state changed most in one step
    (the moving shocks and contacts), at least a block width apart from
    each other and from the blocks already taken."""
    change = np.abs(U_next[0] - U_prev[0]) / np.abs(U_prev[0]).max()
    order = np.argsort(change)[::-1]
    picked = list(taken)
    count += len(picked)
    for i in order[:200000]:
        c = [(int(i) // int(np.prod(n[:d]))) % n[d] for d in range(dim)]
        b = tuple(int(min(max(c[d] - width // 2, 0), n[d] - width)) for d in range(dim))
        if all(max(abs(b[d] - p[d]) for d in range(dim)) >= width for p in picked):
            picked.append(b)
        if len(picked) == count:
            break
    return picked[len(taken):]


LATE = {
    # the schedule's late steps: C2 step 50, C3 step 20
    "2d": dict(make=lambda: W.four_quadrant_state(4096, seed=0), step=50, width=16,
               fixed=[(0, 0), (4080, 4080), (2040, 2040), (0, 2040)], n_active=6,
               n_random=4),
    "3d": dict(make=lambda: W.shock_tube_state(256, seed=0), step=20, width=8,
               fixed=[(0, 0, 0), (248, 248, 248), (120, 0, 124)], n_active=4,
               n_random=2),
}


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("key", ["2d", "3d"])
def test_full_size_late_step(key):
    """The full-size workload stepped by the GPU with its own CFL time steps
    up to step k-1 (k = 50 in 2D, 20 in 3D); from that state the oracle's
    time step on the whole mesh (1e-14), then step k with it on both sides:
    sampled blocks (corners, the most active fronts, seeded interior points)
    against the oracle on windows, and admissibility and conservation of
    mass and total energy since the initial state on the whole field."""
    from oracle import oracle as O
    cfg = LATE[key]
    mesh, U0 = cfg["make"]()
    k = cfg["step"]
    say("late step", key, mesh.n, "build")
    g = abi.Graph(mesh)
    s = abi.Solver(g, gamma=1.4, cfl=0.5)
    s.set_state(U0)
    Uin = s.get_state()
    for _ in range(k - 1):
        s.step_cfl()
    cur = s.get_state()
    say("oracle dt on the whole mesh at step", k - 1)
    og = O.Graph(mesh.dim, mesh.n, mesh.lo, mesh.hi, mesh.periodic, export=False)
    tau = og.compute_dt(O.params(cfl=0.5), cur)
    del og
    t_gpu = s.compute_dt()
    say("dt gpu", t_gpu, "oracle", tau)
    assert t_gpu == pytest.approx(tau, rel=1e-14, abs=0)
    s.step(tau)
    nxt = s.get_state()
    del s

    m = lumped_mass(mesh)
    dim = mesh.dim
    assert np.all(nxt[0] > 0)
    eps = nxt[dim + 1] - 0.5 * (nxt[1:1 + dim] ** 2).sum(axis=0) / nxt[0]
    assert np.all(eps > 0)
    for c in (0, dim + 1):
        a, b = np.dot(m, Uin[c]), np.dot(m, nxt[c])
        assert abs(b - a) <= 1e-12 * abs(a), (c, a, b)

    w = cfg["width"]
    scale = state_scale(cur)
    todo = (list(cfg["fixed"])
            + active_blocks(cur, nxt, dim, mesh.n, w, cfg["n_active"], cfg["fixed"])
            + blocks(mesh, [], cfg["n_random"], w, seed=11))
    # the window oracle projects its input on the walls, which the GPU's
    # state already satisfies to round-off
    for b in todo:
        say("window", b)
        idx, ref = oracle_window_step(mesh, cur, b, (w,) * dim, tau)
        err = state_rel_err(nxt[:, idx], ref, scale=scale)
        say("  err", err.max())
        assert err.max() <= TOL, (key, k, b, err)
