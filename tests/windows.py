"""Oracle results on windows of a large mesh.

One SSPRK(3,3) step at node i depends on the input only within a few nodes
of i (each forward-Euler stage reaches at most 4 neighbours away in
Chebyshev distance: d and alpha one, F^H two, P_ij and pass-1 l three,
pass-2 l four), so the oracle can produce the exact result on a block of
nodes of a mesh far too large for it by running on a sub-mesh that pads
the block with a margin of more than 12 nodes.  Where the margin is cut
from the domain's interior, the sub-mesh has walls there (its coefficients
and slip projection are wrong on those rows), and the damage travels at
most 12 nodes inward per step; where the block touches the true boundary,
the sub-mesh boundary is the true one.  The time step, a global minimum,
is an input, and the bound relaxation uses the whole domain's volume.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2106_02159_amd import workloads as W

MARGIN = 14


def window(mesh: W.Mesh, start, width, margin: int = MARGIN):
    """Sub-mesh around the block [start, start + width) (per direction, node
    indices, clipped to the mesh) and the block's position in it.
    Returns (sub_mesh, full_index, inner) where full_index are the sub-mesh
    nodes' indices in the full mesh (sub-mesh order, x fastest) and inner is
    a boolean mask of the block inside the sub-mesh."""
    assert not any(mesh.periodic), "windows of periodic meshes are not needed"
    dim = mesh.dim
    h = mesh.spacing()
    a0, a1, b0, b1 = [], [], [], []
    for d in range(dim):
        s = max(0, min(int(start[d]), mesh.n[d] - 1))
        e = min(mesh.n[d], s + int(width[d]))
        lo = max(0, s - margin)
        hi = min(mesh.n[d], e + margin)
        a0.append(lo); a1.append(hi); b0.append(s - lo); b1.append(e - lo)
    nw = tuple(a1[d] - a0[d] for d in range(dim))
    sub = W.Mesh(dim, nw,
                 tuple(mesh.lo[d] + a0[d] * h[d] for d in range(dim)),
                 tuple(mesh.lo[d] + (a1[d] - 1) * h[d] for d in range(dim)),
                 (False,) * dim)
    axes = [np.arange(a0[d], a1[d]) for d in range(dim)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]  # x fastest
    full_index = np.zeros(grids[0].shape, np.int64)
    stride = 1
    for d in range(dim):
        full_index += grids[d] * stride
        stride *= mesh.n[d]
    inner = np.ones(grids[0].shape, bool)
    for d in range(dim):
        loc = grids[d] - a0[d]
        inner &= (loc >= b0[d]) & (loc < b1[d])
    return sub, full_index.reshape(-1), inner.reshape(-1)


def volume(mesh: W.Mesh) -> float:
    return float(np.prod([mesh.hi[d] - mesh.lo[d] for d in range(mesh.dim)]))


def oracle_window_step(mesh: W.Mesh, U_full, start, width, tau, prm_kw=None,
                       steps: int = 1):
    """Oracle SSPRK(3,3) steps (slip-projected input, as set_state does) on
    the window around the block; returns (full indices of the block, block
    result (nc, nblock))."""
    sub, idx, inner = window(mesh, start, width, margin=MARGIN * steps)
    g = O.Graph(sub.dim, sub.n, sub.lo, sub.hi, sub.periodic, export=False)
    prm = O.params(volume=volume(mesh), **(prm_kw or {}))
    U = g.slip_bc(U_full[:, idx])
    for _ in range(steps):
        # the status flag (stage CFL check) is not asserted: rows at a cut
        # wall may fail it, and whatever they compute stays in the margin
        U, _ = g.ssprk3_step(prm, U, tau)
    return idx[inner], U[:, inner]
