"""Pins of the oracle's maximum-wave-speed bound (Sec. 3.1) and time step
(Sec. 3.1, eq. dtCfl) against the exact Riemann solution and closed forms."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import riemann_exact as R
from paper_2106_02159_amd import workloads as W

G = 1.4


def _state(rho, vel, p):
    return W.conserved(np.array(rho), tuple(np.array(v) for v in vel), np.array(p), G)


def test_lambda_equal_states():
    rng = np.random.default_rng(3)
    for _ in range(200):
        dim = int(rng.integers(2, 4))
        rho = float(np.exp(rng.uniform(-3, 1)))
        p = float(np.exp(rng.uniform(-3, 1)))
        v = rng.uniform(-2, 2, size=dim)
        n = rng.normal(size=dim)
        n /= np.linalg.norm(n)
        u = _state(rho, v, p)
        lam = O.lambda_max(G, u, u, n)
        ref = abs(v @ n) + math.sqrt(G * p / rho)
        assert lam == pytest.approx(ref, rel=1e-13)


def test_lambda_bounds_exact_riemann_fan():
    """lambda_max dominates the exact extreme wave speeds of the 1D Riemann
    problem (Toro's exact solver), with equality when both waves are
    rarefactions."""
    rng = np.random.default_rng(7)
    n_checked = n_rare = 0
    for _ in range(20000):
        rl, rr = np.exp(rng.uniform(np.log(0.05), np.log(5.0), size=2))
        pl, pr = np.exp(rng.uniform(np.log(0.01), np.log(10.0), size=2))
        ul, ur = rng.uniform(-3, 3, size=2)
        al, ar = math.sqrt(G * pl / rl), math.sqrt(G * pr / rr)
        if 2.0 / (G - 1.0) * (al + ar) <= ur - ul + 1e-9:
            continue  # vacuum
        l1, l3, ps = R.extreme_wave_speeds(rl, ul, pl, rr, ur, pr, G)
        exact = max(-l1, l3, 0.0)
        # embed in 2D along a random direction, tangential velocity arbitrary
        th = rng.uniform(0, 2 * np.pi)
        n = np.array([math.cos(th), math.sin(th)])
        t = np.array([-n[1], n[0]])
        wl, wr = rng.uniform(-1, 1, size=2)
        Ul = _state(rl, ul * n + wl * t, pl)
        Ur = _state(rr, ur * n + wr * t, pr)
        lam = O.lambda_max(G, Ul, Ur, n)
        assert lam >= exact * (1.0 - 1e-12), (lam, exact)
        if ps <= min(pl, pr):
            n_rare += 1
            assert lam == pytest.approx(exact, rel=1e-11)
        n_checked += 1
    assert n_checked > 15000 and n_rare > 500


def test_lambda_mirror_symmetry():
    """Swapping left/right and flipping n describes the same Riemann fan."""
    rng = np.random.default_rng(11)
    for _ in range(500):
        Ui = W.random_rough_state(W.Mesh(3, (1, 1, 1), (0,) * 3, (1,) * 3, (False,) * 3),
                                  seed=int(rng.integers(1 << 30)))[:, 0]
        Uj = W.random_rough_state(W.Mesh(3, (1, 1, 1), (0,) * 3, (1,) * 3, (False,) * 3),
                                  seed=int(rng.integers(1 << 30)))[:, 0]
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        a = O.lambda_max(G, Ui, Uj, n)
        b = O.lambda_max(G, Uj, Ui, -n)
        assert a == pytest.approx(b, rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_dt_closed_form_periodic_rest(dim):
    """Constant state at rest on a periodic mesh: every node is interior and
    lambda_max = a, so tau = c_cfl h / (2 a sum_j |c_ij| / h^(d-1))."""
    n = 6 if dim == 3 else 9
    mesh = W.Mesh(dim, (n,) * dim, (0.0,) * dim, (1.0,) * dim, (True,) * dim)
    rho, p = 1.3, 0.7
    U = W.constant_state(mesh, rho=rho, p=p, gamma=G)
    g = O.Graph(dim, mesh.n, mesh.lo, mesh.hi, mesh.periodic)
    cfl = 0.8
    tau = g.compute_dt(O.params(cfl=cfl), U)
    h = 1.0 / n
    a = math.sqrt(G * p / rho)
    if dim == 2:
        s = (4.0 + math.sqrt(2.0)) / 3.0
    else:
        s = 4.0 / 3.0 + 2.0 * math.sqrt(2.0) / 3.0 + math.sqrt(3.0) / 9.0
    assert tau == pytest.approx(cfl * h / (2.0 * a * s), rel=1e-13)


def test_dt_scales_with_cfl():
    mesh, U = W.four_quadrant_state(12, seed=1)
    g = O.Graph(2, mesh.n, mesh.lo, mesh.hi, mesh.periodic)
    t1 = g.compute_dt(O.params(cfl=1.0), U)
    t2 = g.compute_dt(O.params(cfl=0.25), U)
    assert t2 == pytest.approx(0.25 * t1, rel=1e-15)
