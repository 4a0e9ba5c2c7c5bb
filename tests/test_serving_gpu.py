"""Serving (continuous batching of independent simulations): asynchronous
steps equal synchronous ones bit for bit; the footprint estimate equals the
allocation; the server admits by memory and never exceeds its budget;
every request's result is bit-identical alone and in the mix."""
import time

import numpy as np
import pytest

from paper_2106_02159_amd import abi, workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precision", [abi.PREC_FP64, abi.PREC_MIXED])
def test_footprint_equals_allocation(precision):
    for mesh, _ in (W.four_quadrant_state(67, seed=0), W.shock_tube_state(9, seed=0),
                    (W.Mesh(2, (33, 20), (0, 0), (1, 1), (True, False)), None)):
        g = abi.Graph(mesh)
        s = abi.Solver(g, precision=precision)
        assert abi.footprint(g, precision=precision) == s.device_bytes()


def test_async_steps_equal_sync_steps():
    mesh, U = W.four_quadrant_state(97, seed=4)
    g = abi.Graph(mesh)
    a = abi.Solver(g)
    a.set_state(U)
    t_sync = sum(a.step_cfl() for _ in range(7))
    b = abi.Solver(g)
    b.set_state(U)
    b.step_cfl_async(3)
    b.step_cfl_async(4)
    while not b.query():
        time.sleep(1e-3)
    rc, t_async = b.async_finish()
    assert rc == abi.NS_OK
    assert t_async == pytest.approx(t_sync, rel=1e-15)
    assert np.array_equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("dim,precision", [(2, abi.PREC_FP64), (3, abi.PREC_FP64),
                                           (2, abi.PREC_MIXED)])
def test_graph_replays_equal_eager_steps(dim, precision):
    """Asynchronous steps replay a captured graph of one step per start
    buffer; every replay, with eager work and host synchronisation between
    them, equals the eagerly launched synchronous steps bit for bit."""
    mesh, U = (W.four_quadrant_state(75, seed=5) if dim == 2
               else W.shock_tube_state(14, seed=5))
    g = abi.Graph(mesh)
    a = abi.Solver(g, precision=precision)
    b = abi.Solver(g, precision=precision)
    a.set_state(U)
    b.set_state(U)
    for rnd in range(4):
        say("graph replay round", rnd, "dim", dim, "precision", precision)
        t_sync = a.step_cfl() + a.step_cfl() + a.step_cfl()
        b.step_cfl_async(2)
        b.step_cfl_async(1)
        rc, t_async = b.async_finish()
        assert rc == abi.NS_OK
        assert t_async == t_sync
        assert np.array_equal(a.get_state(), b.get_state())
        # eager work on b between replays: a profiled (eager) step and back
        b.profile(True)
        b.step_cfl()
        b.profile(False)
        a.step_cfl()
        assert np.array_equal(a.get_state(), b.get_state())


def run_server(reqs, mem_bytes, max_running, precision=abi.PREC_FP64, stagger=0.0,
               pack_nodes=0, pack_max=64, persistent_rows=0):
    sv = abi.Server(mem_bytes, max_running=max_running, precision=precision,
                    pack_nodes=pack_nodes, pack_max=pack_max,
                    persistent_rows=persistent_rows)
    ids = []
    for mesh, U, steps in reqs:
        ids.append(sv.submit(mesh, U, steps))
        sv.progress()
        if stagger:
            time.sleep(stagger)
    left = set(ids)
    out = {}
    t0 = time.time()
    while left:
        sv.progress()
        for rid in list(left):
            if sv.request(rid).state == abi.REQ_FINISHED:
                info = sv.request(rid)
                U, st = sv.result(rid)
                assert st == abi.NS_OK, sv.error(rid)
                out[rid] = (U, info.t_sim)
                left.discard(rid)
        assert time.time() - t0 < 120, "server did not finish"
        time.sleep(1e-3)
    st = sv.stats()
    sv.close()
    return [out[r] for r in ids], st


def mix(count=6, steps=12, seed=0):
    reqs = []
    for k, n in enumerate([48, 131, 64, 160, 77, 100][:count]):
        mesh, U = W.four_quadrant_state(n, seed=seed + k)
        reqs.append((mesh, U, steps))
    return reqs


@pytest.mark.parametrize("precision", [abi.PREC_FP64, abi.PREC_MIXED])
def test_alone_and_in_the_mix_are_identical(precision):
    reqs = mix()
    alone = []
    for r in reqs:
        res, _ = run_server([r], 1 << 34, 1, precision)
        alone.append(res[0])
    together, st = run_server(reqs, 1 << 34, 6, precision, stagger=0.002)
    say("peak running", st.peak_running)
    assert st.peak_running >= 2
    for (ua, ta), (ub, tb) in zip(alone, together):
        assert np.array_equal(ua, ub)
        assert ta == tb
    # and equal to a plain solver run
    mesh, U, steps = reqs[1]
    s = abi.Solver(abi.Graph(mesh), precision=precision)
    s.set_state(U)
    for _ in range(steps):
        s.step_cfl()
    assert np.array_equal(s.get_state(), together[1][0])


@pytest.mark.parametrize("precision", [abi.PREC_FP64, abi.PREC_MIXED])
def test_packed_requests_equal_alone(precision):
    """With packs (up to 65536 rows, 4 members): the six requests run as two
    packs of consecutive requests (4 + 2 members); every result and its
    simulated time are bit-identical to the request run alone."""
    reqs = mix()
    alone = [run_server([r], 1 << 34, 1, precision)[0][0] for r in reqs]
    packed, st = run_server(reqs, 1 << 34, 6, precision, pack_nodes=65536, pack_max=4)
    say("peak running", st.peak_running)
    assert st.finished == len(reqs)
    for (ua, ta), (ub, tb) in zip(alone, packed):
        assert np.array_equal(ua, ub)
        assert ta == tb
    # requests with another step count are not packed with them
    reqs2 = reqs[:3] + [(reqs[3][0], reqs[3][1], 7)] + reqs[4:]
    packed2, _ = run_server(reqs2, 1 << 34, 6, precision, pack_nodes=65536, pack_max=4)
    solo3, _ = run_server([reqs2[3]], 1 << 34, 1, precision)
    assert np.array_equal(packed2[3][0], solo3[0][0])
    for k in (0, 1, 2, 4, 5):
        assert np.array_equal(packed2[k][0], alone[k][0])


def test_pack_admission_by_memory():
    """A pack shrinks to the members whose pack footprint fits the memory
    left; every request still finishes."""
    reqs = [(*W.four_quadrant_state(60, seed=k), 6) for k in range(6)]
    g = [abi.Graph(m) for m, _, _ in reqs]
    budget = abi.pack_footprint(g[:3])
    res, st = run_server(reqs, budget, 8, pack_nodes=1 << 20, pack_max=64)
    say("peak running", st.peak_running, "peak bytes", st.peak_bytes, "budget", budget)
    assert st.finished == 6
    assert st.peak_bytes <= budget
    assert st.peak_running == 3


def test_inadmissible_request_is_refused_at_submission():
    (m, U), (m2, U2) = W.four_quadrant_state(30, seed=1), W.four_quadrant_state(31, seed=2)
    sv = abi.Server(1 << 34, pack_nodes=1 << 20)
    bad = U.copy()
    bad[-1, 17] = 0.999 * 0.5 * (bad[1, 17] ** 2 + bad[2, 17] ** 2) / bad[0, 17]  # eps < 0
    with pytest.raises(abi.NSError) as ex:
        sv.submit(m, bad, 3)
    assert ex.value.code == abi.NS_ENOTADMISSIBLE
    rid = sv.submit(m2, U2, 3)
    while sv.request(rid).state != abi.REQ_FINISHED:
        sv.progress()
    out, st = sv.result(rid)
    assert st == abi.NS_OK
    sv.close()


@pytest.mark.parametrize("pack_nodes", [0, 1 << 20])
def test_zero_steps_returns_the_projected_state(pack_nodes):
    reqs = [(*W.four_quadrant_state(40, seed=3), 0), (*W.four_quadrant_state(41, seed=4), 0)]
    res, st = run_server(reqs, 1 << 34, 4, pack_nodes=pack_nodes)
    for (mesh, U, _), (out, t) in zip(reqs, res):
        s = abi.Solver(abi.Graph(mesh))
        s.set_state(U)
        assert t == 0.0
        assert np.array_equal(out, s.get_state())


def test_admission_by_memory():
    reqs = [(*W.four_quadrant_state(90, seed=k), 10) for k in range(5)]
    fp = abi.footprint(abi.Graph(reqs[0][0]))
    res, st = run_server(reqs, int(2.5 * fp), 16)
    say("peak running", st.peak_running, "peak bytes", st.peak_bytes, "budget", 2.5 * fp)
    assert st.peak_running == 2
    assert st.peak_bytes <= 2.5 * fp
    assert st.finished == 5
    # a request larger than the budget is refused at submission
    sv = abi.Server(fp // 2)
    with pytest.raises(abi.NSError):
        sv.submit(reqs[0][0], reqs[0][1], 3)
    sv.close()
