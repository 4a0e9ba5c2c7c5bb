"""ns_stats_noalloc through the C ABI: the same statistics as ns_stats,
computed with the library's fixed device scratch instead of a per-call
allocation.  Two calls in a row, the second on a smaller mesh, each equal
to ns_stats field by field (the reductions are deterministic)."""
import ctypes as C

import pytest

from paper_2106_02159_amd import abi, workloads as W

pytestmark = pytest.mark.gpu

FIELDS = [f for f, _ in abi.Stats._fields_]


def noalloc_stats(s):
    """ns_stats_noalloc called through the C ABI."""
    out = abi.Stats()
    rc = abi.lib().ns_stats_noalloc(s.h, C.byref(out))
    assert rc == abi.NS_OK, abi.lib().ns_last_error(s.h)
    return out


def stepped(make, steps, **kw):
    mesh, U = make()
    s = abi.Solver(abi.Graph(mesh), cfl=0.5, **kw)
    s.set_state(U)
    for _ in range(steps):
        s.step_cfl()
    return s


@pytest.mark.parametrize("mixed", [False, True])
def test_noalloc_matches_stats(mixed):
    prec = dict(precision=abi.PREC_MIXED if mixed else abi.PREC_FP64)
    # 640^2 rows need more workgroups than the scratch has partial slots
    # (the kernels stride), then a smaller mesh, then a 3D one
    for make, steps in ((lambda: W.four_quadrant_state(640, seed=1), 2),
                        (lambda: W.four_quadrant_state(96, seed=2), 3),
                        (lambda: W.shock_tube_state(20, seed=0), 2)):
        s = stepped(make, steps, **prec)
        b = noalloc_stats(s)
        a = s.stats()
        for f in FIELDS:
            assert getattr(a, f) == getattr(b, f), (f, getattr(a, f), getattr(b, f))
        assert a.limited1 > 0 and a.min_rho > 0
        s.close()


def test_noalloc_errors():
    fn = abi.lib().ns_stats_noalloc
    mesh, U = W.four_quadrant_state(16, seed=0)
    s = abi.Solver(abi.Graph(mesh))
    out = abi.Stats()
    assert fn(s.h, C.byref(out)) == abi.NS_ESTATE  # no state yet
    assert fn(None, C.byref(out)) == abi.NS_EINVAL
    s.set_state(U)
    assert fn(s.h, None) == abi.NS_EINVAL
