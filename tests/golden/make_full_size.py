"""Writes full_size_dt.json: the oracle's time step for the two full-size
workloads (2D four-quadrant data on 4096x4096 nodes, 3D Mach-3 shock tube on
256^3 nodes, seed 0, c_cfl = 0.5, gamma = 1.4), computed from the
slip-projected initial state as tau = c_cfl min_i m_i / (2 sum_j d_ij)
(time-step rule of Sec. 3.1).

The full-size parity tests feed this tau to the library's step and compare
windows of the result with the oracle run on sub-meshes; tau itself is a
global minimum over all nodes, which a window cannot see, so it is computed
here once on the whole mesh.  Only oracle/ and the seeded workload
generators are used.  Needs about 45 GB of host memory for the 3D mesh.

usage: python tests/golden/make_full_size.py [2d] [3d]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2106_02159_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "full_size_dt.json")

CASES = {
    "2d": ("four_quadrant", 4096),
    "3d": ("shock_tube", 256),
}


def oracle_dt(kind: str, n: int, seed: int = 0) -> float:
    if kind == "four_quadrant":
        mesh, U = W.four_quadrant_state(n, seed=seed)
    else:
        mesh, U = W.shock_tube_state(n, seed=seed)
    g = O.Graph(mesh.dim, mesh.n, mesh.lo, mesh.hi, mesh.periodic, export=False)
    U = g.slip_bc(U)
    return g.compute_dt(O.params(cfl=0.5), U)


def main():
    which = sys.argv[1:] or list(CASES)
    O.build(force=False)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for key in which:
        kind, n = CASES[key]
        t0 = time.perf_counter()
        tau = oracle_dt(kind, n)
        data[key] = {"workload": kind, "n": n, "seed": 0, "cfl": 0.5,
                     "gamma": 1.4, "tau": tau}
        print(f"{key}: tau = {tau!r} ({time.perf_counter() - t0:.1f} s)", flush=True)
    data["_source"] = ("tests/golden/make_full_size.py: oracle compute_dt on the "
                       "slip-projected seed-0 initial state (time-step rule, Sec. 3.1)")
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
