"""Persistent steps (ns_step_cfl_persistent): whole SSPRK(3,3) steps with
the CFL time step as one kernel launch whose workgroups take (step, stage,
phase, member, row block) items in order.  Checked: bit-identity with the
launch-based asynchronous steps (2D and 3D, FP64 and mixed precision,
meshes whose last row block is ragged, runs that mix both kinds of call);
pack members equal their own solvers; the server gives the same results
with persistent launches, alone and in the mix; the bounded waits give up
when the host sets the give-up word or the wait limit is reached, every
workgroup exits, the run reports NS_EABORT and the solver works again
after a new state is set."""
import time

import numpy as np
import pytest

from paper_2106_02159_amd import abi, workloads as W
from tests.test_serving_gpu import mix, run_server

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def finish(s):
    while not s.query():
        time.sleep(1e-3)
    return s.async_finish()


def state(dim, n, seed):
    return W.four_quadrant_state(n, seed=seed) if dim == 2 else W.shock_tube_state(n, seed=seed)


@pytest.mark.parametrize("dim,n,precision", [(2, 100, abi.PREC_FP64), (2, 100, abi.PREC_MIXED),
                                             (2, 64, abi.PREC_FP64), (3, 20, abi.PREC_FP64),
                                             (3, 17, abi.PREC_MIXED)])
def test_persistent_equals_launched_steps(dim, n, precision):
    """n = 100 (2D) and 20, 17 (3D) leave a ragged last row block."""
    mesh, U = state(dim, n, 3)
    g = abi.Graph(mesh)
    a = abi.Solver(g, precision=precision)
    b = abi.Solver(g, precision=precision)
    a.set_state(U)
    b.set_state(U)
    say("persistent vs launched", dim, n, precision)
    a.step_cfl_async(3)
    a.step_cfl_async(2)
    rca, ta = finish(a)
    b.step_cfl_persistent(3)
    b.step_cfl_persistent(2)
    rcb, tb = finish(b)
    assert rca == rcb == abi.NS_OK
    assert ta == tb
    assert np.array_equal(a.get_state(), b.get_state())


def test_mixed_calls_in_one_run():
    mesh, U = W.four_quadrant_state(90, seed=7)
    g = abi.Graph(mesh)
    a = abi.Solver(g)
    a.set_state(U)
    t_sync = sum(a.step_cfl() for _ in range(6))
    b = abi.Solver(g)
    b.set_state(U)
    b.step_cfl_async(2)
    b.step_cfl_persistent(1)
    b.step_cfl_async(1)
    b.step_cfl_persistent(2)
    rc, t = finish(b)
    assert rc == abi.NS_OK and t == t_sync
    assert np.array_equal(a.get_state(), b.get_state())
    # a second run on the same solver
    for _ in range(2):
        a.step_cfl()
    b.step_cfl_persistent(2)
    rc, _ = finish(b)
    assert rc == abi.NS_OK
    assert np.array_equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("dim,precision", [(2, abi.PREC_FP64), (2, abi.PREC_MIXED),
                                           (3, abi.PREC_FP64)])
def test_pack_members_equal_own_solvers(dim, precision):
    """Members of different sizes (so different row-block, work-list and
    slip-slice counts), one of them periodic (no slip nodes)."""
    if dim == 2:
        items = [W.four_quadrant_state(n, seed=k) for k, n in enumerate((64, 100, 37))]
        items.append((W.Mesh(2, (40, 70), (0, 0), (1, 1), (True, False)), None))
        items.append(W.vortex_state(48))
    else:
        items = [W.shock_tube_state(n, seed=k) for k, n in enumerate((12, 17, 9))]
    mems = []
    for mesh, U in items:
        if U is None:
            _, U0 = W.four_quadrant_state(mesh.n[0], seed=9)
            U = np.stack([np.resize(c, mesh.N) for c in U0])
        mems.append((mesh, U))
    graphs = [abi.Graph(m) for m, _ in mems]
    pk = abi.Pack(graphs, precision=precision)
    for r, (_, U) in enumerate(mems):
        pk.set_state(r, U)
    say("pack persistent", dim, precision, [g.N for g in graphs])
    pk.step_cfl_persistent(2)
    pk.step_cfl_persistent(3)
    st, t = pk.finish()
    assert all(x == abi.NS_OK for x in st)
    for r, (g, (_, U)) in enumerate(zip(graphs, mems)):
        s = abi.Solver(g, precision=precision)
        s.set_state(U)
        tt = sum(s.step_cfl() for _ in range(5))
        assert t[r] == tt
        assert np.array_equal(pk.get_state(r), s.get_state()), r


@pytest.mark.parametrize("precision", [abi.PREC_FP64, abi.PREC_MIXED])
def test_server_persistent_alone_and_in_the_mix(precision):
    reqs = mix()
    launched, _ = run_server(reqs, 1 << 34, 6, precision, stagger=0.002,
                             pack_nodes=65536, pack_max=4)
    alone = [run_server([r], 1 << 34, 1, precision, persistent_rows=1 << 40)[0][0]
             for r in reqs]
    together, st = run_server(reqs, 1 << 34, 6, precision, stagger=0.002, pack_nodes=65536,
                              pack_max=4, persistent_rows=1 << 40)
    say("peak running", st.peak_running, "units", st.units)
    for (ua, ta), (ub, tb), (uc, tc) in zip(alone, together, launched):
        assert np.array_equal(ua, ub) and np.array_equal(ub, uc)
        assert ta == tb == tc


def test_wait_limit_gives_up_and_solver_recovers():
    mesh, U = W.four_quadrant_state(200, seed=1)
    g = abi.Graph(mesh)
    s = abi.Solver(g)
    s.set_state(U)
    say("wait limit 1 ns")
    s.step_cfl_persistent(2, wait_s=1e-9)
    s.step_cfl_persistent(1, wait_s=10.0)  # stopped too: the stop is sticky
    rc, _ = finish(s)
    assert rc == abi.NS_EABORT
    with pytest.raises(abi.NSError) as ei:
        s.step_cfl()
    assert ei.value.code == abi.NS_ESTATE
    # a new state: both kinds of steps work again and agree
    s.set_state(U)
    ref = abi.Solver(g)
    ref.set_state(U)
    ref.step_cfl_async(2)
    assert finish(ref)[0] == abi.NS_OK
    s.step_cfl_persistent(2)
    assert finish(s)[0] == abi.NS_OK
    assert np.array_equal(s.get_state(), ref.get_state())


def test_cancel_stops_the_launches_in_flight():
    mesh, U = W.four_quadrant_state(1024, seed=2)
    g = abi.Graph(mesh)
    s = abi.Solver(g)
    s.set_state(U)
    say("cancel of 2 x 20 steps on 1024^2")
    s.step_cfl_persistent(20)
    s.step_cfl_persistent(20)
    s.cancel()
    t0 = time.time()
    rc, _ = finish(s)
    say("finished after", time.time() - t0, "s")
    assert rc == abi.NS_EABORT
    s.set_state(U)
    s.step_cfl_persistent(1)
    assert finish(s)[0] == abi.NS_OK
    # packs: the same through ns_pack_cancel
    pk = abi.Pack([g, abi.Graph(W.four_quadrant_state(300, seed=3)[0])])
    pk.set_state(0, U)
    pk.set_state(1, W.four_quadrant_state(300, seed=3)[1])
    pk.step_cfl_persistent(20)
    pk.cancel()
    st, _ = pk.finish()
    assert st == [abi.NS_EABORT, abi.NS_EABORT]


def test_unsupported_configurations_are_refused():
    mesh, U = W.four_quadrant_state(40, seed=0)
    g = abi.Graph(mesh)
    for kw in ({"limiter": abi.LIM_LOW}, {"passes": 1}, {"indicator": abi.IND_ONE}):
        s = abi.Solver(g, **kw)
        s.set_state(U)
        with pytest.raises(abi.NSError) as ei:
            s.step_cfl_persistent(1)
        assert ei.value.code == abi.NS_EINVAL
    s = abi.Solver(g)
    s.set_state(U)
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(abi.NSError):
            s.step_cfl_persistent(1, wait_s=bad)
    with pytest.raises(abi.NSError):
        abi.Server(1 << 30, persistent_rows=-1)
