"""The window method used by the full-size parity tests, checked on meshes
the oracle can run whole: the oracle on a window (block + margin) must give
the whole-mesh oracle's result on the block, at corners, walls, the interior
and across the workloads' discontinuities, for one and for two steps."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2106_02159_amd import workloads as W
from tests.helpers import state_rel_err, state_scale
from tests.windows import oracle_window_step

CASES = [
    ("quad2d", lambda: W.four_quadrant_state(96, seed=0), 8,
     [(0, 0), (88, 88), (44, 0), (0, 40), (44, 44), (20, 60)]),
    ("tube3d", lambda: W.shock_tube_state(40, seed=0), 4,
     [(0, 0, 0), (8, 18, 18), (8, 0, 18), (36, 36, 36), (18, 4, 30)]),
]


@pytest.mark.parametrize("name,make,w,starts", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("steps", [1, 2])
def test_window_matches_whole_mesh(name, make, w, starts, steps):
    mesh, U0 = make()
    g = O.Graph(mesh.dim, mesh.n, mesh.lo, mesh.hi, mesh.periodic, export=False)
    prm = O.params()
    U = g.slip_bc(U0)
    tau = g.compute_dt(prm, U)
    full = U
    for _ in range(steps):
        full, _ = g.ssprk3_step(prm, full, tau)
    for s in starts:
        idx, blk = oracle_window_step(mesh, U0, s, (w,) * mesh.dim, tau, steps=steps)
        err = state_rel_err(blk, full[:, idx], scale=state_scale(full))
        assert err.max() <= 1e-13, (name, s, err)
