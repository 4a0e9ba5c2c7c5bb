"""GPU parity with the strict local bounds of Sec. 3.3 (bound relaxation
r0 = 0): the admissible set of the line search is exactly
[rho_min, rho_max] x {Phi >= Phi_min} built from the bar states and the
neighbours' specific entropies, with no widening.

With strict bounds the limiter's output is not a well-conditioned function
of its input wherever the entropy bound is tight: in isentropic flow Phi is
constant, so Phi(U^L) - Phi_min is rounding noise, the sign of the
line-search function psi near l = 0 is decided by that noise, and the step's
result moves by up to 1e-9..1e-7 (relative) when the input moves by 1e-15.
No independent implementation can then agree with the oracle to 1e-12.
So each comparison here measures the oracle's own sensitivity first -- the
oracle rerun on the same input with a seeded relative perturbation of
1e-15 -- and requires

    |GPU - oracle| <= max(TOL_FLOOR, 10 * sensitivity)

relative to the field's max norm, per component.  TOL_FLOOR = 1e-11 covers
the root of psi itself: where psi is flat its computed sign changes over a
band of l wider than round-off, and the two root finders (the oracle's
bisection, the GPU's Newton iteration with a feasibility check) may return
different feasible points inside that band (measured: 4.8e-12 on the 3D
shock tube, whose oracle sensitivity is 3e-15).  Rough states (node-wise
random data) hold 1e-15 here, like the relaxed default."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2106_02159_amd import abi, workloads as W
from tests.helpers import rel_err, state_rel_err
from tests.test_parity_gpu import CASES

pytestmark = pytest.mark.gpu

TOL_FLOOR = 1e-11
NOISE = 1e-15


def say(*a):
    print(*a, flush=True)


def perturbed(U, seed):
    rng = np.random.default_rng(seed)
    return U * (1.0 + NOISE * rng.uniform(-1.0, 1.0, U.shape))


def tolerance(ref, ref_pert):
    """Per-component bar: the floor or ten times the oracle's own response
    to input noise, whichever is larger."""
    sens = state_rel_err(ref_pert, ref)
    return np.maximum(TOL_FLOOR, 10.0 * sens), sens


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    mesh, U = CASES[request.param]()
    og = O.Graph(mesh.dim, mesh.n, mesh.lo, mesh.hi, mesh.periodic)
    U = og.slip_bc(U)
    return request.param, mesh, og, abi.Graph(mesh), U


def test_stage_strict(case):
    """One forward-Euler stage with strict bounds; the bounds themselves
    (no relaxation) to 1e-13 and the stage result to the bar above."""
    name, mesh, og, g, U = case
    prm = O.params(cfl=0.9, relax=0.0)
    tau = og.compute_dt(prm, U)
    ref, st, dbg = og.fe_stage(prm, U, tau, debug=True)
    ref_p, _, _ = og.fe_stage(prm, perturbed(U, 1), tau, debug=True)
    tol, sens = tolerance(ref, ref_p)
    s = abi.Solver(g, cfl=0.9, relax=0.0)
    s.set_state(U, project=False)
    assert s.fe_stage(tau) == abi.NS_OK, abi.lib().ns_last_error(s.h)
    assert np.all(rel_err(s.debug("bounds"), dbg["bounds"], axis=1) <= 1e-13)
    err = state_rel_err(s.debug("stage_out"), ref)
    say("strict stage", name, "err", err.max(), "oracle sensitivity", sens.max())
    assert np.all(err <= tol), (name, err, tol)


def test_step_strict(case):
    """Two SSPRK(3,3) steps with strict bounds, each from the GPU's state."""
    name, mesh, og, g, U = case
    prm = O.params(cfl=0.9, relax=0.0)
    s = abi.Solver(g, cfl=0.9, relax=0.0)
    s.set_state(U, project=False)
    cur = U
    for k in range(2):
        tau = og.compute_dt(prm, cur)
        ref, st = og.ssprk3_step(prm, cur, tau)
        assert st == 0
        ref_p, _ = og.ssprk3_step(prm, perturbed(cur, 10 + k), tau)
        tol, sens = tolerance(ref, ref_p)
        s.set_state(cur, project=False)
        s.step(tau)
        cur = s.get_state()
        err = state_rel_err(cur, ref)
        say("strict step", name, k + 1, "err", err.max(), "oracle sensitivity", sens.max())
        assert np.all(err <= tol), (name, k, err, tol)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_four_quadrant_strict(seed):
    """Four-quadrant data on 256x256 with walls and strict bounds: steps 1, 2
    and 20, each from the GPU's own state; conservation of mass and energy
    over all 20 steps."""
    mesh, U = W.four_quadrant_state(256, seed=seed)
    og = O.Graph(2, mesh.n, mesh.lo, mesh.hi, mesh.periodic)
    prm = O.params(cfl=0.5, relax=0.0)
    s = abi.Solver(abi.Graph(mesh), cfl=0.5, relax=0.0)
    s.set_state(U)
    U0 = s.get_state()
    for k in range(20):
        cur = s.get_state()
        tau = og.compute_dt(prm, cur)
        if k in (0, 1, 19):
            ref, st = og.ssprk3_step(prm, cur, tau)
            assert st == 0
            ref_p, _ = og.ssprk3_step(prm, perturbed(cur, 100 + k), tau)
            tol, sens = tolerance(ref, ref_p)
            s.step(tau)
            err = state_rel_err(s.get_state(), ref)
            say("strict quad256 seed", seed, "step", k + 1, "err", err.max(),
                "oracle sensitivity", sens.max())
            assert np.all(err <= tol), (seed, k, err, tol)
        else:
            s.step(tau)
    out = s.get_state()
    for c in (0, 3):
        a, b = (og.mi * U0[c]).sum(), (og.mi * out[c]).sum()
        assert abs(a - b) <= 1e-13 * abs(a)
    eps = out[3] - 0.5 * (out[1] ** 2 + out[2] ** 2) / out[0]
    assert np.all(out[0] > 0) and np.all(eps > 0)


def test_vortex_strict():
    """Isentropic vortex (periodic 64x64, CFL 0.5) with strict bounds: the
    ill-conditioned case (Phi constant); 10 steps, every one compared from
    the GPU's own state to the sensitivity bar."""
    mesh, U = W.vortex_state(64)
    og = O.Graph(2, mesh.n, mesh.lo, mesh.hi, mesh.periodic)
    prm = O.params(cfl=0.5, relax=0.0)
    s = abi.Solver(abi.Graph(mesh), cfl=0.5, relax=0.0)
    s.set_state(U)
    worst = 0.0
    for k in range(10):
        cur = s.get_state()
        tau = og.compute_dt(prm, cur)
        ref, st = og.ssprk3_step(prm, cur, tau)
        ref_p, _ = og.ssprk3_step(prm, perturbed(cur, 200 + k), tau)
        tol, sens = tolerance(ref, ref_p)
        s.step(tau)
        err = state_rel_err(s.get_state(), ref)
        worst = max(worst, err.max())
        assert np.all(err <= tol), (k, err, tol, sens)
    say("strict vortex64 10 steps, worst error", worst)
