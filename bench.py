"""Throughput of the explicit hyperbolic step (SSPRK(3,3) with convex
limiting) on one MI355X.

One benchmark step = one SSPRK(3,3) step of the whole hot path: the time
step computed on the device from the first stage's graph viscosity, three
forward-Euler stages (graph viscosity, indicator, low-order update, bounds,
high-order flux, two limiter passes) and the slip post-processing after
each stage.  Workload: 2D Euler, gamma = 1.4, Q1 on a 4096x4096-node uniform
mesh of [0,1]^2 with reflecting walls, seeded four-quadrant Riemann data, FP64
(--dim 3: the 3D Mach-3 shock tube on 256^3 nodes, the hyperbolic step of the
Navier-Stokes configuration).
Metric: DoF-updates per second per SSP-RK stage = nodes x 3 x steps / time.

Prints one JSON line.  --gpus above 1 is not supported (one GPU per run).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2106_02159_amd import abi, workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per node per launch of each kernel (sliced ELL edge
# arrays; column indices, m_ij and c_ij derived from the box mesh, not moved;
# every array a kernel touches counted once; W = 3^d slots, nc = d + 2
# components).  With `mixed`, alpha, d_ij, F^H and the limiter coefficients
# are 4-byte values; everything else is FP64.
def kernel_bytes(name: str, dim: int, mixed: bool = False) -> float:
    Wd = 3 ** dim
    nc = dim + 2
    na = dim + 5
    L = 4 if mixed else 8          # storage of the FP32-capable arrays
    # column indices, m_ij and c_ij are derived from the box mesh, not loaded
    eL = L * Wd                    # one per-edge array (d, l)
    n8, nL = 8, L
    rows = nc * (2 * n8 + nL)      # U, U^L (or U^(1)) and F^H of the row
    table = {
        "prim": nc * n8 + (na - dim - 1) * n8,  # U -> a, b, eta, Phi
        "visc": nc * n8 + 3 * n8 + 1 + eL + nL,  # U, a, b, eta (v, p from U)
        "visc_dt": (dim + 3) * n8 + 1 + eL,
        "dt_partial": eL + n8,
        "lo": eL + nc * n8 + 1 * n8 + nL + 3 * n8  # U, Phi (v, p from U), alpha, ...
              + nc * n8 + nc * nL + 3 * n8,
        "lim1": eL + rows + nL + 2 * n8 + 3 * n8 + eL,
        "lim2": (2 * eL + rows + nL + 2 * n8 + 3 * n8 + nc * n8 + eL
                 if dim == 2 else  # 3D: pass-1 update only
                 2 * eL + rows + nL + 2 * n8 + nc * n8),
        "lim2b": 2 * eL + rows + nL + 2 * n8 + 3 * n8 + eL,
        "fin": 2 * eL + nc * (3 * n8 + nL) + nL + 2 * n8 + nc * n8,
        "combine": 2 * nc * n8 + nc * n8,
        "slip": 0.0,
        "dt_final": 0.0,
    }
    return float(table.get(name, 0.0))


def stage_algorithmic_bytes(dim: int, mixed: bool = False) -> float:
    """Bytes per node per forward-Euler stage if m_i and the state were each
    moved once (the column indices, m_ij and c_ij follow from the box mesh):
    read U, write the stage result, read U^n in two of the three stages;
    93 B in 2D, 115 B in 3D, in either precision mode."""
    nc = dim + 2
    return 8 + 2 * 8 * nc + 8 * nc * 2 / 3


def source_sha() -> str:
    """sha256 (first 16 hex) of the device code and its launch code:
    csrc/*.hip and *.hpp (the host-only *.cpp files -- graph and element
    tables, the server -- do not change what a kernel moves)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_02159_amd", "csrc")
    for ext in ("hip", "hpp"):
        for p in sorted(glob.glob(os.path.join(csrc, f"*.{ext}"))):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, tag: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of workload `tag`, or None if the kernel sources changed since it
    was taken."""
    path = os.path.join(ROOT, "profiles", f"hyp_stage_{tag}_hbm_traffic.md")
    try:
        txt = open(path).read()
        data = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if data.get("source_sha") != source_sha():
        return None
    k = data.get("kernels", {}).get(kernel)
    return k["traffic_bytes"] if k else None


def workload(dim: int, n: int, seed: int):
    if dim == 2:
        return W.four_quadrant_state(n, seed=seed)
    return W.shock_tube_state(n, seed=seed)


def cpu_baseline(dim: int, n_sample: int, seed: int, ns: bool = False,
                 min_s: float = 10.0, max_steps: int = 16, mu: float = 1e-4):
    """The oracle, as it stands, stepping the same workload at n_sample
    nodes per direction: SSPRK(3,3) steps (Strang steps with `ns`), each with
    its CFL time step, until at least min_s seconds have passed (at most
    max_steps steps; graph assembly not timed)."""
    from oracle import oracle as O
    O.build(force=False)
    mesh, U = workload(dim, n_sample, seed)
    og = O.Graph(dim, mesh.n, mesh.lo, mesh.hi, mesh.periodic, export=False)
    prm = O.params(cfl=0.5)
    visc = O.visc(mu=mu, lam=0.0, kappa=1.4 * mu, cv=2.5, cg_rtol=1e-10, cg_maxit=20000)
    U = og.slip_bc(U)
    steps = 0
    t0 = time.perf_counter()
    while True:
        tau = og.compute_dt(prm, U)
        if ns:
            U, st, _ = og.strang_step(prm, visc, U, tau)
        else:
            U, st = og.ssprk3_step(prm, U, tau)
        if st != 0:
            raise RuntimeError(f"oracle step failed with status {st}")
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or steps >= max_steps:
            break
    stages = 6 if ns else 3
    what = (f"{steps} Strang steps (time step + 6 stages + parabolic step each; "
            f"the oracle's parabolic part is serial)" if ns else
            f"{steps} SSPRK3 steps (time step + 3 stages each)")
    return {"value": og.N * stages * steps / dt, "unit": "DoF-updates/s per SSP-RK stage",
            "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{what} of the "
                      f"{'four-quadrant' if dim == 2 else 'Mach-3 shock-tube'} "
                      f"workload at {n_sample}^{dim} nodes, seed {seed}, "
                      f"{dt:.2f} s"}


def serve_bench(args):
    """Serving workload: `requests` independent four-quadrant problems, N x N
    nodes with N log-uniform in [64, 1024], `serve_steps` SSPRK(3,3) steps
    each, Poisson arrivals at `rate` per second, admitted by device-memory
    footprint; reports request latency (submission to completion)
    percentiles and the whole-job throughput."""
    prec = abi.PREC_MIXED if args.mixed else abi.PREC_FP64
    reqs = W.serving_requests(args.requests, seed=args.seed, rate=args.rate)
    states = [W.four_quadrant_state(n, seed=sd) for _, n, sd in reqs]
    mem = int(args.serve_mem_gb * 2 ** 30)
    # warm-up: one small request through a server (first HIP use, module load)
    warm = abi.Server(mem, max_running=1, precision=prec)
    wid = warm.submit(states[0][0], states[0][1], 2)
    while warm.request(wid).state != abi.REQ_FINISHED:
        warm.progress()
        time.sleep(1e-3)
    warm.close()
    sv = abi.Server(mem, max_running=args.max_running, precision=prec,
                    chunk=args.serve_chunk, depth=2, pack_nodes=args.pack_nodes,
                    pack_max=args.pack_max)
    t0 = time.perf_counter()
    pending = list(range(len(reqs)))
    ids, info = {}, {}
    t_progress = 0.0
    while len(info) < len(reqs):
        now = time.perf_counter() - t0
        while pending and reqs[pending[0]][0] <= now:
            k = pending.pop(0)
            ids[sv.submit(states[k][0], states[k][1], args.serve_steps)] = k
        tp = time.perf_counter()
        sv.progress()
        t_progress += time.perf_counter() - tp
        for rid in list(ids):
            r = sv.request(rid)
            if r.state == abi.REQ_FINISHED:
                _, st = sv.result(rid)
                if st != abi.NS_OK:
                    raise RuntimeError(f"request {ids[rid]} failed: {sv.error(rid)}")
                info[ids.pop(rid)] = (r.t_submit, r.t_finish, r.n_nodes)
        time.sleep(2e-4)
    stats = sv.stats()
    sv.close()
    lat = np.array([f - s for s, f, _ in info.values()]) * 1e3
    t_first = min(s for s, _, _ in info.values())
    t_last = max(f for _, f, _ in info.values())
    dof = sum(n for _, _, n in info.values()) * 3 * args.serve_steps
    value = dof / (t_last - t_first)
    return {
        "metric": "DoF-updates/s per SSP-RK stage; p50/p99 request latency",
        "value": value,
        "unit": "DoF-updates/s per SSP-RK stage",
        "n_gpus": 1, "steps": args.serve_steps, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (f32 storage)" if args.mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} independent 2D Euler Q1 requests, "
                               f"N x N nodes with N log-uniform in [64, 1024], seeded "
                               f"four-quadrant data, {args.serve_steps} SSPRK3 steps "
                               f"each, Poisson arrivals at {args.rate}/s, admission by "
                               f"device footprint (budget {args.serve_mem_gb} GiB, at "
                               f"most {args.max_running} running units), requests "
                               f"of at most {args.pack_nodes // 2} rows packed "
                               f"(consecutive, same step count, up to "
                               f"{args.pack_nodes} rows and {args.pack_max} members "
                               f"per pack), chunks of {args.serve_chunk} steps, "
                               f"{args.hw_queues} hardware queues",
                   "requests": args.requests},
        "latency_ms": {"p50": float(np.percentile(lat, 50)),
                       "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "max": float(lat.max())},
        "makespan_s": t_last - t_first,
        "host_progress_s": t_progress,
        "peak_running": stats.peak_running,
        "peak_bytes": stats.peak_bytes,
        "units": stats.units,
        "host_s": {"admit": stats.host_admit_s, "top_up": stats.host_topup_s,
                   "finish": stats.host_finish_s},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3),
                    help="2: four-quadrant data on 4096^2 nodes; 3: Mach-3 "
                         "shock tube on 256^3 nodes (hyperbolic step)")
    ap.add_argument("--n", type=int, default=0,
                    help="nodes per direction (default 4096 in 2D, 256 in 3D)")
    ap.add_argument("--ns", action="store_true",
                    help="Navier-Stokes: Strang steps (hyperbolic tau, parabolic "
                         "2 tau, hyperbolic tau) with mu = 1e-4, lambda = 0, "
                         "kappa = 1.4e-4, cv = 1/(gamma-1), CG rtol 1e-10")
    ap.add_argument("--mu", type=float, default=1e-4,
                    help="Navier-Stokes: shear viscosity (kappa = 1.4 mu)")
    ap.add_argument("--precond", choices=("jacobi", "gmg"), default="jacobi",
                    help="Navier-Stokes: preconditioner of the parabolic CG (gmg: "
                         "FP32 multigrid V-cycle, for the viscous-dominated regime)")
    ap.add_argument("--mixed", action="store_true",
                    help="mixed precision: FP32 storage of alpha, d_ij, F^H and "
                         "the limiter coefficients, "
                         "FP64 state and arithmetic; after the timed steps the FP64 "
                         "path is run with the same time steps and the L1 relative "
                         "error is reported")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload (continuous batching of independent "
                         "requests); prints latency percentiles and throughput")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--serve-steps", type=int, default=200)
    ap.add_argument("--max-running", type=int, default=8,
                    help="serving: running units (solvers or packs) at most")
    ap.add_argument("--serve-mem-gb", type=float, default=160.0)
    ap.add_argument("--serve-chunk", type=int, default=2,
                    help="steps per enqueued chunk of a running request")
    ap.add_argument("--pack-nodes", type=int, default=1 << 21,
                    help="serving: rows of a pack of small requests at most (0: "
                         "every request gets its own solver)")
    ap.add_argument("--pack-max", type=int, default=64,
                    help="serving: members of a pack at most")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues for the serving streams (GPU_MAX_HW_QUEUES, "
                         "at most 32)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle sample, nodes per direction (default 1024 in "
                         "2D, 96 in 3D)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the hyperbolic step is benchmarked "
              "on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        # set before the first HIP call of the process; the running requests'
        # streams are spread over these hardware queues
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(max(args.hw_queues, 1), 32))
        print(json.dumps(serve_bench(args)), flush=True)
        return
    dim = 3 if args.ns else args.dim
    n = args.n or (4096 if dim == 2 else 256)
    t0 = time.perf_counter()
    mesh, U = workload(dim, n, args.seed)
    graph = abi.Graph(mesh)
    solver = abi.Solver(graph, gamma=1.4, cfl=0.5,
                        precision=abi.PREC_MIXED if args.mixed else abi.PREC_FP64)
    solver.set_state(U)
    del U
    if args.ns:
        solver.set_viscous(mu=args.mu, lam=0.0, kappa=1.4 * args.mu, cv=1.0 / 0.4,
                           cg_rtol=1e-10, cg_maxit=20000,
                           precond=abi.PC_GMG if args.precond == "gmg" else abi.PC_JACOBI)
        advance = solver.step_strang_cfl
    else:
        advance = solver.step_cfl
    setup_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        advance()
    solver.sync()
    solver.profile(True)
    solver.sync()
    cg_iters = []
    taus = []
    U_warm = solver.get_state() if args.mixed else None
    solver.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        taus.append(advance())
        if args.ns:
            info = solver.parabolic_info()
            cg_iters.append((info.it_v, info.it_e, info.it_l, info.fct))
    solver.sync()
    elapsed = time.perf_counter() - t0
    rep = solver.profile_report()
    solver.profile(False)
    roots = solver.debug("roots")
    # plain device copy of 1 GiB: the achievable streaming bandwidth, and a
    # kernel of known traffic for calibrating hardware byte counters
    copy_bytes = 1 << 30
    copy_ms = solver.copy_bench(copy_bytes, reps=5, word=16)
    copy_gbs = 2 * copy_bytes / (copy_ms * 1e-3) / 1e9
    copy8_ms = solver.copy_bench(copy_bytes, reps=5, word=8)
    copy8_gbs = 2 * copy_bytes / (copy8_ms * 1e-3) / 1e9

    N = graph.N
    stages_per_step = 6 if args.ns else 3
    stages = stages_per_step * args.steps
    value = N * stages / elapsed
    tag = f"{dim}d_{n}" + ("_mixed" if args.mixed else "") + ("_ns" if args.ns else "")
    # dominant kernel by summed time
    dom = max(rep.items(), key=lambda kv: kv[1][1])
    dname, (dlaunch, dms) = dom
    avg_s = dms / dlaunch * 1e-3
    kb = kernel_bytes(dname, dim, args.mixed) * N
    achieved = kb / avg_s / 1e9
    kern = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1),
                "algorithmic_GBs": kernel_bytes(k, dim, args.mixed) * N
                / (v[1] / max(v[0], 1) * 1e-3) / 1e9
                if kernel_bytes(k, dim, args.mixed) > 0 else None}
            for k, v in rep.items()}
    stage_frac = stage_algorithmic_bytes(dim, args.mixed) * value / (HBM_PEAK_GBS * 1e9)
    out = {
        "metric": "DoF-updates/s per SSP-RK stage",
        "value": value,
        "unit": "DoF-updates/s per SSP-RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (
                       f"3D Navier-Stokes gamma=1.4, Q1 {n}^3 nodes on [0,1]^3, "
                       f"mu={args.mu:g}, lambda=0, kappa={1.4 * args.mu:g}, cv=2.5, "
                       f"Mach-3 shock tube with seeded 1% density noise (seed "
                       f"{args.seed}); Strang step = SSPRK3(tau) + parabolic CN/CG(2 tau, "
                       f"{'multigrid V-cycle (FP32, Chebyshev(3)-Jacobi)' if args.precond == 'gmg' else 'Jacobi'}, "
                       f"rtol 1e-10; no-slip, insulated walls) + SSPRK3(tau), CFL 0.5"
                       if args.ns else
                       f"2D Euler gamma=1.4, Q1 {n}x{n} nodes on [0,1]^2, "
                       f"reflecting walls, seeded four-quadrant Riemann data "
                       f"(seed {args.seed}), SSPRK3 + 2-pass convex limiting, CFL 0.5"
                       + (", mixed precision (FP32 storage of alpha, d_ij, F^H, "
                          "limiter coefficients)" if args.mixed else "")
                       if dim == 2 else
                       f"3D Euler gamma=1.4 (hyperbolic step of the Navier-Stokes "
                       f"configuration), Q1 {n}^3 nodes on [0,1]^3, reflecting walls, "
                       f"Mach-3 shock tube with seeded 1% density noise (seed "
                       f"{args.seed}), SSPRK3 + 2-pass convex limiting, CFL 0.5"),
                   "nodes": N, "stages_per_step": stages_per_step},
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dname, tag),
                     "algorithmic_bytes": kb},
        "stage_algorithmic_frac": stage_frac,
        "copy_GBs": copy_gbs,
        "copy8_GBs": copy8_gbs,
        "kernels": kern,
        "root_edges_last_stage": {"pass1": int(roots[0]), "pass2": int(roots[1]),
                                  "edges": int(graph.nnz - N)},
        "setup_s": setup_s,
        "device_bytes": solver.device_bytes(),
    }
    if args.mixed:
        # the FP64 path (parity-tested against the oracle) from the same state
        # with the same time steps
        U_mp = solver.get_state()
        solver.close()
        ref = abi.Solver(graph, gamma=1.4, cfl=0.5, precision=abi.PREC_FP64)
        ref.set_state(U_warm, project=False)
        for t in taus:
            ref.step(t)
        U_64 = ref.get_state()
        ref.close()
        nrm = lambda a: float(np.abs(a).sum())
        out["error_vs_fp64"] = {
            "rho": nrm(U_mp[0] - U_64[0]) / nrm(U_64[0]),
            "m": nrm(U_mp[1:1 + dim] - U_64[1:1 + dim]) / nrm(U_64[1:1 + dim]),
            "E": nrm(U_mp[dim + 1] - U_64[dim + 1]) / nrm(U_64[dim + 1]),
            "steps": args.steps, "norm": "L1 relative",
            "reference": "the FP64 path of this library on the same time steps"}
        out["dtype"] = "f64 (f32 storage)"
    if args.ns:
        out["cg_iterations"] = {"velocity": [c[0] for c in cg_iters],
                                "energy": [c[1] for c in cg_iters],
                                "low_order": [c[2] for c in cg_iters],
                                "limited_steps": sum(c[3] for c in cg_iters)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(
            dim, args.cpu_sample or (1024 if dim == 2 else (64 if args.ns else 96)),
            args.seed, ns=args.ns, mu=args.mu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
