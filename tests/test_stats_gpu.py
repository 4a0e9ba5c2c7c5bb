"""ns_stats through the C ABI: admissibility minima of the current state and
the limiter activity of the last stage, checked against the oracle's state
and intermediates and against the library's own debug arrays."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2106_02159_amd import abi, workloads as W
from tests.helpers import ell_to_csr_index

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def eps_of(U):
    dim = U.shape[0] - 2
    return U[dim + 1] - 0.5 * (U[1:1 + dim] ** 2).sum(axis=0) / U[0]


def host_counts(s, g):
    """Pass-1 and pass-2 limited entries recounted on the host from the
    library's own stage arrays (ELL, both directions of every entry)."""
    ex = g.export()
    col = ex["col"]
    Wd, N = col.shape
    lt1, lt2 = s.debug("lt1"), s.debug("lt2")
    rows = np.broadcast_to(np.arange(N), col.shape)
    mask = (col >= 0) & (col != rows)
    k, i = np.nonzero(mask)
    j = col[k, i]
    kt = Wd - 1 - k
    l = np.minimum(lt1[k, i], lt1[kt, j])
    w = np.minimum(lt2[k, i], lt2[kt, j])
    return int(mask.sum()), int((l < 1).sum()), int((l + w < 1).sum())


@pytest.mark.parametrize("mixed", [False, True])
def test_stats_after_steps(mixed):
    """Four-quadrant data on 130x130 after 3 steps: min rho / min eps equal
    the state's own minima and agree with the oracle's state of the same
    steps (1e-12); the limited counts equal the host recount of the stage
    arrays; the root counts equal NS_DBG_ROOTS."""
    mesh, U = W.four_quadrant_state(130, seed=2)
    og = O.Graph(2, mesh.n, mesh.lo, mesh.hi, mesh.periodic)
    prm = O.params(cfl=0.5)
    g = abi.Graph(mesh)
    s = abi.Solver(g, cfl=0.5, precision=abi.PREC_MIXED if mixed else abi.PREC_FP64)
    cur = og.slip_bc(U)
    s.set_state(cur, project=False)
    for _ in range(3):
        tau = og.compute_dt(prm, cur)
        cur, st = og.ssprk3_step(prm, cur, tau)
        assert st == 0
        s.step(tau)
    st = s.stats()
    out = s.get_state()
    e = eps_of(out)
    assert st.min_rho == out[0].min() and out[0, st.argmin_rho] == st.min_rho
    assert st.argmin_rho == int(np.argmin(out[0]))
    assert st.min_eps == pytest.approx(e.min(), rel=1e-15)
    assert st.argmin_eps == int(np.argmin(e)) or e[st.argmin_eps] == e.min()
    tol = 1e-6 if mixed else 1e-12
    assert st.min_rho == pytest.approx(cur[0].min(), rel=tol)
    assert st.min_eps == pytest.approx(eps_of(cur).min(), rel=tol)
    edges, c1, c2 = host_counts(s, g)
    say("stats", "mixed" if mixed else "fp64", "edges", st.edges, "limited", st.limited1,
        st.limited2, "roots", st.roots1, st.roots2)
    assert st.edges == edges == g.nnz - g.N
    assert (st.limited1, st.limited2) == (c1, c2)
    assert 0 < st.limited2 <= st.limited1 < edges
    roots = s.debug("roots")
    assert (st.roots1, st.roots2) == (int(roots[0]), int(roots[1]))
    assert st.cg_it_v == st.cg_it_e == st.fct == 0


def test_stats_stage_vs_oracle():
    """One forward-Euler stage on quad67: the limited counts agree with the
    oracle's symmetric limiters of the same stage, except for entries whose
    oracle value lies within the 1e-10 parity band of 1."""
    mesh, U = W.four_quadrant_state(67, seed=1)
    og = O.Graph(2, mesh.n, mesh.lo, mesh.hi, mesh.periodic)
    U = og.slip_bc(U)
    prm = O.params(cfl=0.9)
    tau = og.compute_dt(prm, U)
    _, st, dbg = og.fe_stage(prm, U, tau, debug=True)
    g = abi.Graph(mesh)
    s = abi.Solver(g, cfl=0.9)
    s.set_state(U, project=False)
    s.fe_stage(tau)
    stt = s.stats()
    rows = np.repeat(np.arange(og.N), np.diff(og.row_ptr))
    off = og.col != rows
    l1, l2 = dbg["l1"][off], dbg["l2"][off]
    tot = l1 + l2 * (1.0 - l1)
    band = 1e-10
    assert np.sum(l1 < 1 - band) <= stt.limited1 <= np.sum(l1 < 1)
    assert np.sum(tot < 1 - band) <= stt.limited2 <= np.sum(tot < 1 + band)
    assert stt.edges == off.sum()
    # the state is the one set (a stage does not change it)
    assert stt.min_rho == U[0].min()


def test_stats_modes_and_parabolic():
    """Without convex limiting the limiter fields are -1; one pass leaves
    limited2 / roots2 at -1; after a Strang step the CG counts are those of
    ns_parabolic_info."""
    mesh, U = W.four_quadrant_state(40, seed=5)
    g = abi.Graph(mesh)
    s = abi.Solver(g, limiter=abi.LIM_LOW)
    s.set_state(U)
    st0 = s.stats()  # before any stage
    assert st0.limited1 == st0.limited2 == st0.roots1 == st0.roots2 == -1
    s.step_cfl()
    st = s.stats()
    assert st.limited1 == st.limited2 == -1 and st.min_rho > 0 and st.min_eps > 0
    s1 = abi.Solver(g, passes=1)
    s1.set_state(U)
    s1.step_cfl()
    st1 = s1.stats()
    assert st1.limited1 >= 0 and st1.roots1 >= 0 and st1.limited2 == -1 and st1.roots2 == -1
    mesh3, U3 = W.shock_tube_state(10, seed=0)
    s3 = abi.Solver(abi.Graph(mesh3))
    s3.set_state(U3)
    s3.set_viscous(mu=1e-3, lam=0.0, kappa=1.4e-3, cv=2.5, cg_rtol=1e-12)
    s3.step_strang_cfl()
    info = s3.parabolic_info()
    st3 = s3.stats()
    assert (st3.cg_it_v, st3.cg_it_e, st3.cg_it_l, st3.fct) == (info.it_v, info.it_e,
                                                               info.it_l, info.fct)
    assert st3.cg_it_v > 0 and st3.min_eH == info.min_eH
