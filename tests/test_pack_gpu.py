"""Packs: several meshes advanced by the same kernel launches, each member
with its own CFL time step and status.  Every member's result equals that
of its own solver (ns_step_cfl) bit for bit, and the oracle's step with the
member's time step to the step bar.  Members span one workgroup exactly,
ragged tails, periodic and tiny meshes (mostly padding rows)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2106_02159_amd import abi, workloads as W
from tests.helpers import state_rel_err

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rough(mesh, seed):
    return mesh, W.random_rough_state(mesh, seed=seed)


def members(dim):
    if dim == 2:
        return [W.four_quadrant_state(48, seed=1),        # 2304 rows: 9 workgroups
                W.four_quadrant_state(67, seed=2),        # ragged tail
                rough(W.Mesh(2, (40, 23), (0, 0), (1.0, 0.6), (True, False)), 3),
                rough(W.Mesh(2, (2, 2), (0, 0), (1, 1), (False, False)), 4),
                W.vortex_state(32)]
    return [W.shock_tube_state(9, seed=1), W.shock_tube_state(12, seed=2),
            rough(W.Mesh(3, (7, 5, 6), (0,) * 3, (1.0, 0.7, 0.9), (False, True, False)), 3)]


@pytest.mark.parametrize("dim,precision", [(2, abi.PREC_FP64), (3, abi.PREC_FP64),
                                           (2, abi.PREC_MIXED)])
def test_members_equal_their_own_solvers(dim, precision):
    ms = members(dim)
    graphs = [abi.Graph(m) for m, _ in ms]
    pk = abi.Pack(graphs, precision=precision)
    for r, (m, U) in enumerate(ms):
        pk.set_state(r, U)
    say("pack", dim, precision, [g.N for g in graphs])
    pk.step_cfl_async(2)
    pk.step_cfl_async(3)
    st, t = pk.finish()
    assert st == [abi.NS_OK] * len(ms)
    for r, (m, U) in enumerate(ms):
        s = abi.Solver(graphs[r], precision=precision)
        s.set_state(U)
        tt = 0.0
        for _ in range(5):
            tt += s.step_cfl()
        assert t[r] == tt, (r, t[r], tt)
        assert np.array_equal(pk.get_state(r), s.get_state()), r
    # the next run starts its time and status afresh
    pk.step_cfl_async(1)
    st, t2 = pk.finish()
    assert st == [abi.NS_OK] * len(ms) and np.all(t2 > 0) and np.all(t2 < t)
    pk.close()


def test_member_step_matches_oracle():
    ms = members(2)
    graphs = [abi.Graph(m) for m, _ in ms]
    pk = abi.Pack(graphs)
    for r, (m, U) in enumerate(ms):
        pk.set_state(r, U)
    pk.step_cfl_async(1)
    st, t = pk.finish()
    assert st == [abi.NS_OK] * len(ms)
    prm = O.params(cfl=0.5)
    for r, (m, U) in enumerate(ms):
        og = O.Graph(m.dim, m.n, m.lo, m.hi, m.periodic)
        U0 = og.slip_bc(U)
        assert t[r] == pytest.approx(og.compute_dt(prm, U0), rel=1e-14, abs=0)
        ref, rc = og.ssprk3_step(prm, U0, t[r])
        assert rc == 0
        err = state_rel_err(pk.get_state(r), ref)
        say("member", r, "err", err.max())
        assert np.all(err <= 1e-12), (r, err)
    pk.close()


def test_pack_errors():
    (m2, U2), (m3, U3) = W.four_quadrant_state(20, seed=0), W.shock_tube_state(6, seed=0)
    g2, g3 = abi.Graph(m2), abi.Graph(m3)
    with pytest.raises(abi.NSError):
        abi.Pack([g2, g3])          # members of different dimensions
    with pytest.raises(abi.NSError):
        abi.Pack([])
    pk = abi.Pack([g2, abi.Graph(W.four_quadrant_state(30, seed=1)[0])])
    pk.set_state(0, U2)
    with pytest.raises(abi.NSError) as ex:
        pk.step_cfl_async(1)        # member 1 has no state yet
    assert ex.value.code == abi.NS_ESTATE
    bad = U2.copy()
    bad[0, 7] = -1.0
    with pytest.raises(abi.NSError) as ex:
        pk.set_state(0, bad)
    assert ex.value.code == abi.NS_ENOTADMISSIBLE
    with pytest.raises(abi.NSError):
        pk.finish()                 # nothing enqueued
    pk.close()
