"""Throughput of the explicit hyperbolic step (SSPRK(3,3) with convex
limiting) on one MI355X, and the configurations around it.

One benchmark step = one SSPRK(3,3) step of the whole hot path: the time
step computed on the device from the first stage's graph viscosity, three
forward-Euler stages (graph viscosity, indicator, low-order update, bounds,
high-order flux, two limiter passes) and the slip post-processing after
each stage.  Headline workload (the JSON line's metric and value): 2D Euler,
gamma = 1.4, Q1 on a 4096x4096-node uniform mesh of [0,1]^2 with reflecting
walls, seeded four-quadrant Riemann data, FP64, CFL 0.5.
Metric: DoF-updates per second per SSP-RK stage = nodes x 3 x steps / time.

The default run also measures, in the same process and reported under
"configs": the 3D Mach-3 shock tube on 256^3 nodes (hyperbolic step, and
the Navier-Stokes Strang step), the 4096^2 workload in mixed precision with
its L1 difference from the FP64 path after 50 steps, and the serving
workload (256 requests, Poisson arrivals) in FP64 and mixed precision with
p50/p99 latency.  --dim 3 / --ns / --mixed / --serve run one of these alone
(as the headline), which is how the profiles are taken.

Roofline: the algorithmic bytes per node per forward-Euler stage of the
method with its graph stored as the paper stores it (column index, c_ij,
m_ij, m_i, the state read and written, U^n for the SSP combination: 345 B in
2D with 9-point rows, 1087 B in 3D with 27-point rows) times the nodes,
divided by the stage's duration -- the sum of its kernels' HIP-event times
on the solver's stream -- against the 8 TB/s HBM peak.

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

# Algorithmic bytes per node per forward-Euler stage with the graph stored
# (FP64; 2D: col 36 + c_ij 144 + m_ij 72 + m_i 8 + U read 32 + U written 32
# + U^n in two of three stages 21; 3D: 108 + 648 + 216 + 8 + 40 + 40 + 27).
STAGE_BYTES = {2: 345.0, 3: 1087.0}


# Algorithmic bytes per node per launch of each kernel of this design (sliced
# ELL edge arrays; column indices, m_ij and c_ij derived from the box mesh,
# not moved; every array a kernel touches counted once; W = 3^d slots,
# nc = d + 2 components).  With `mixed`, alpha, d_ij, F^H and the limiter
# coefficients are 4-byte values; everything else is FP64.
def kernel_bytes(name: str, dim: int, mixed: bool = False) -> float:
    Wd = 3 ** dim
    nc = dim + 2
    na = dim + 5
    L = 4 if mixed else 8          # storage of the FP32-capable arrays
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
        # 2D: both pass-1 searches, the update and the pass-2 search in one
        # sweep (d, the row's U, U^L, F^H, alpha, m_i, lambda_i, bounds in;
        # l~, U^(1), l~' out); the deferred rows are a small fraction
        "lim12": 3 * eL + rows + nL + 2 * n8 + 3 * n8 + nc * n8,
        "lim2d": 0.0,
        "fin": 2 * eL + nc * (3 * n8 + nL) + nL + 2 * n8 + nc * n8,
        "combine": 2 * nc * n8 + nc * n8,
        "slip": 0.0,
        "dt_final": 0.0,
    }
    return float(table.get(name, 0.0))


def source_sha() -> str:
    """sha256 (first 16 hex) of the device code and its launch code:
    csrc/*.hip and *.hpp except the host driver ns_api.hip (it allocates,
    uploads and sequences the launches whose kernels and grids the other
    files define; like the host-only *.cpp files -- graph and element
    tables, the server -- it does not change what a kernel moves)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_02159_amd", "csrc")
    for ext in ("hip", "hpp"):
        for p in sorted(glob.glob(os.path.join(csrc, f"*.{ext}"))):
            if os.path.basename(p) == "ns_api.hip":
                continue
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(tag: str):
    """Per-kernel HBM bytes per launch from the committed rocprofv3 counter
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
    return {k: v["traffic_bytes"] for k, v in data.get("kernels", {}).items()}


def workload(dim: int, n: int, seed: int):
    if dim == 2:
        return W.four_quadrant_state(n, seed=seed)
    return W.shock_tube_state(n, seed=seed)


def workload_name(dim, n, seed, mixed=False, ns=False, mu=1e-4, precond="jacobi"):
    if ns:
        return (f"3D Navier-Stokes gamma=1.4, Q1 {n}^3 nodes on [0,1]^3, "
                f"mu={mu:g}, lambda=0, kappa={1.4 * mu:g}, cv=2.5, "
                f"Mach-3 shock tube with seeded 1% density noise (seed {seed}); "
                f"Strang step = SSPRK3(tau) + parabolic CN/CG(2 tau, "
                + ("multigrid V-cycle (FP32, Chebyshev(3)-Jacobi)" if precond == "gmg"
                   else "Jacobi")
                + ", rtol 1e-10; no-slip, insulated walls) + SSPRK3(tau), CFL 0.5")
    if dim == 2:
        return (f"2D Euler gamma=1.4, Q1 {n}x{n} nodes on [0,1]^2, reflecting walls, "
                f"seeded four-quadrant Riemann data (seed {seed}), SSPRK3 + 2-pass "
                f"convex limiting, CFL 0.5"
                + (", mixed precision (FP32 storage of alpha, d_ij, F^H, limiter "
                   "coefficients)" if mixed else ""))
    return (f"3D Euler gamma=1.4 (hyperbolic step of the Navier-Stokes configuration), "
            f"Q1 {n}^3 nodes on [0,1]^3, reflecting walls, Mach-3 shock tube with "
            f"seeded 1% density noise (seed {seed}), SSPRK3 + 2-pass convex limiting, "
            f"CFL 0.5")


PRECISIONS = (abi.PREC_FP64, abi.PREC_MIXED, abi.PREC_MIXED_FP32)


def run_steps(graph, U, dim, mixed, steps, warmup, ns=False, mu=1e-4, precond="jacobi"):
    """Time `steps` CFL steps (Strang steps with `ns`) of one solver on the
    state U after `warmup` untimed ones; mixed: 0 FP64, 1 FP32 storage, 2
    FP32 storage and FP32 evaluation.  Returns a dict of results."""
    solver = abi.Solver(graph, gamma=1.4, cfl=0.5, precision=PRECISIONS[int(mixed)])
    solver.set_state(U)
    if ns:
        solver.set_viscous(mu=mu, lam=0.0, kappa=1.4 * mu, cv=1.0 / 0.4, cg_rtol=1e-10,
                           cg_maxit=20000,
                           precond=abi.PC_GMG if precond == "gmg" else abi.PC_JACOBI)
        advance = solver.step_strang_cfl
    else:
        advance = solver.step_cfl
    for _ in range(warmup):
        advance()
    solver.sync()
    solver.profile(True)
    solver.sync()
    cg, taus = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        taus.append(advance())
        if ns:
            info = solver.parabolic_info()
            cg.append((info.it_v, info.it_e, info.it_l, info.fct))
    solver.sync()
    elapsed = time.perf_counter() - t0
    rep = solver.profile_report()
    solver.profile(False)
    roots = solver.debug("roots")
    st = solver.stats()
    N = graph.N
    stages = (6 if ns else 3) * steps
    value = N * stages / elapsed
    # the whole stage: every kernel it launches (HIP events on the solver's
    # stream), per forward-Euler stage; parabolic kernels excluded
    par = ("par_", "cg_")
    hyp = {k: v for k, v in rep.items() if not k.startswith(par)}
    stage_ms = sum(v[1] for v in hyp.values()) / stages
    kern = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1),
                "per_stage": v[0] / stages,
                "algorithmic_GBs": kernel_bytes(k, dim, mixed) * N
                / (v[1] / max(v[0], 1) * 1e-3) / 1e9
                if kernel_bytes(k, dim, mixed) > 0 else None}
            for k, v in rep.items()}
    out = {
        "solver": solver, "value": value, "elapsed": elapsed,
        "ms_per_step": elapsed / steps * 1e3, "stage_ms": stage_ms, "kernels": kern,
        "taus": taus, "cg": cg, "roots": roots, "stats": st, "N": N,
        "device_bytes": solver.device_bytes(),
    }
    return out


def stage_roofline(res, dim, tag):
    """The roofline object of a run: the whole forward-Euler stage against
    the algorithmic bytes per node (STAGE_BYTES), and the measured per-stage
    HBM bytes from the committed counter summary of the same workload."""
    N = res["N"]
    algo = STAGE_BYTES[dim] * N
    achieved = algo / (res["stage_ms"] * 1e-3) / 1e9
    traffic = None
    per_kernel = measured_traffic(tag)
    if per_kernel is not None:
        traffic = 0.0
        for k, v in res["kernels"].items():
            if k.startswith(("par_", "cg_")):
                continue  # the parabolic step is not part of the stage
            if k in per_kernel:
                traffic += per_kernel[k] * v["per_stage"]
            elif k not in ("slip", "dt_final", "nonreflecting"):
                traffic = None
                break
    return {"bound": "hbm", "kernel": "stage", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_node": STAGE_BYTES[dim],
            "traffic_bytes_per_node": traffic / N if traffic is not None else None,
            "stage_ms": res["stage_ms"],
            "frac_wallclock": res["value"] * STAGE_BYTES[dim] / (HBM_PEAK_GBS * 1e9)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(O, dim, n, seed, max_steps, min_s, ns=False, mu=1e-4, vortex=False):
    """The oracle stepping a workload at n nodes per direction: SSPRK(3,3)
    steps (Strang steps with `ns`), each with its CFL time step, until
    min_s seconds have passed or max_steps steps are done (graph assembly
    not timed).  Returns (DoF-updates/s per stage, steps, seconds, N)."""
    if vortex:
        mesh, U = W.vortex_state(n)
    else:
        mesh, U = workload(dim, n, seed)
    og = O.Graph(mesh.dim, mesh.n, mesh.lo, mesh.hi, mesh.periodic, export=False)
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
    return og.N * stages * steps / dt, steps, dt, og.N


def cpu_baseline(dim: int, n_sample: int, seed: int, ns: bool = False,
                 min_s: float = 10.0, max_steps: int = 16, mu: float = 1e-4,
                 single: bool = True):
    """The oracle, as it stands, on the host cores: all of them on a sample
    of the workload (n_sample nodes per direction, until min_s seconds), and
    with `single` also one core on one whole step of that sample and on the
    whole isentropic-vortex configuration (64^2 periodic nodes, 100 steps)."""
    from oracle import oracle as O
    O.build(force=False)
    nthreads = O.num_threads()
    v, steps, dt, N = oracle_rate(O, dim, n_sample, seed, max_steps, min_s, ns=ns, mu=mu)
    kind = "Strang" if ns else "SSPRK3"
    name = "four-quadrant" if dim == 2 else "Mach-3 shock-tube"
    out = {"value": v, "unit": "DoF-updates/s per SSP-RK stage", "cores": nthreads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{steps} {kind} steps (time step + {6 if ns else 3} stages each"
                     + ("; the oracle's parabolic part is serial" if ns else "")
                     + f") of the {name} workload at {n_sample}^{dim} nodes, seed {seed}, "
                     f"{dt:.2f} s on {nthreads} threads"}
    if single:
        O.set_num_threads(1)
        try:
            v1, s1, d1, _ = oracle_rate(O, dim, n_sample, seed, 1, 0.0, ns=ns, mu=mu)
            vv, sv, dv, Nv = oracle_rate(O, 2, 64, 0, 100, 1e9, vortex=True)
        finally:
            O.set_num_threads(nthreads)
        out["single_core"] = {
            "value": v1, "cores": 1,
            "sample": f"one {kind} step of the {name} workload at {n_sample}^{dim} nodes, "
                      f"{d1:.2f} s"}
        out["vortex_single_core"] = {
            "value": vv, "cores": 1,
            "sample": f"the whole isentropic-vortex configuration: {sv} SSPRK3 steps at "
                      f"CFL 0.5 on the periodic 64x64 mesh, {dv:.2f} s"}
    return out


def serve_bench(args, mixed: bool):
    """Serving workload: `requests` independent four-quadrant problems, N x N
    nodes with N log-uniform in [64, 1024], `serve_steps` SSPRK(3,3) steps
    each, Poisson arrivals at `rate` per second, admitted by device-memory
    footprint; reports request latency (submission to completion)
    percentiles and the whole-job throughput."""
    prec = abi.PREC_MIXED if mixed else abi.PREC_FP64
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
                    pack_max=args.pack_max, persistent_rows=args.persistent_rows)
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
    offered = sum(n * n for _, n, _ in reqs) * 3 * args.serve_steps / reqs[-1][0]
    return {
        "value": dof / (t_last - t_first),
        "unit": "DoF-updates/s per SSP-RK stage",
        "dtype": "f64 (f32 storage)" if mixed else "f64",
        "workload": f"serving: {args.requests} independent 2D Euler Q1 requests, "
                    f"N x N nodes with N log-uniform in [64, 1024], seeded "
                    f"four-quadrant data, {args.serve_steps} SSPRK3 steps "
                    f"each, Poisson arrivals at {args.rate}/s, admission by "
                    f"device footprint (budget {args.serve_mem_gb} GiB, at "
                    f"most {args.max_running} running units), requests "
                    f"of at most {args.pack_nodes // 2} rows packed "
                    f"(consecutive, same step count, up to "
                    f"{args.pack_nodes} rows and {args.pack_max} members "
                    f"per pack), chunks of {args.serve_chunk} steps "
                    + (f"(one persistent launch per chunk for units of at most "
                       f"{args.persistent_rows} rows, captured step graphs above), "
                       if args.persistent_rows > 0 else "(captured step graphs), ")
                    + f"{args.hw_queues} hardware queues",
        "requests": args.requests,
        "latency_ms": {"p50": float(np.percentile(lat, 50)),
                       "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "max": float(lat.max())},
        "offered_load": offered,
        "makespan_s": t_last - t_first,
        "host_progress_s": t_progress,
        "peak_running": stats.peak_running,
        "peak_bytes": stats.peak_bytes,
        "units": stats.units,
        "host_s": {"admit": stats.host_admit_s, "top_up": stats.host_topup_s,
                   "finish": stats.host_finish_s},
    }


def base_line(metric, value, steps, warmup, ms_per_step, dtype, config):
    return {"metric": metric, "value": value, "unit": "DoF-updates/s per SSP-RK stage",
            "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config}


def copy_bandwidth(solver):
    """A plain device copy of 1 GiB: the achievable streaming bandwidth, and
    a kernel of known traffic for calibrating the hardware byte counters."""
    copy_bytes = 1 << 30
    ms16 = solver.copy_bench(copy_bytes, reps=5, word=16)
    ms8 = solver.copy_bench(copy_bytes, reps=5, word=8)
    return {"copy_GBs": 2 * copy_bytes / (ms16 * 1e-3) / 1e9,
            "copy8_GBs": 2 * copy_bytes / (ms8 * 1e-3) / 1e9}


def summary(res, dim, tag, extra=None):
    st = res["stats"]
    d = {"value": res["value"], "ms_per_step": res["ms_per_step"],
         "roofline": stage_roofline(res, dim, tag),
         "min_rho": st.min_rho, "min_eps": st.min_eps,
         "limited_fraction": {"pass1": st.limited1 / st.edges if st.limited1 >= 0 else None,
                              "pass2": st.limited2 / st.edges if st.limited2 >= 0 else None},
         "root_edges_last_stage": {"pass1": int(res["roots"][0]),
                                   "pass2": int(res["roots"][1])},
         "device_bytes": res["device_bytes"]}
    if extra:
        d.update(extra)
    return d


def mixed_error(graph, U0, steps, dim, precision=abi.PREC_MIXED):
    """Mixed precision against the FP64 path (itself parity-tested against
    the oracle) after `steps` CFL steps from the same state with the mixed
    run's time steps: L1 relative difference of rho, m, E; admissibility of
    the mixed result."""
    mp = abi.Solver(graph, gamma=1.4, cfl=0.5, precision=precision)
    mp.set_state(U0)
    taus = [mp.step_cfl() for _ in range(steps)]
    U_mp = mp.get_state()
    st = mp.stats()
    mp.close()
    ref = abi.Solver(graph, gamma=1.4, cfl=0.5, precision=abi.PREC_FP64)
    ref.set_state(U0)
    for t in taus:
        ref.step(t)
    U_64 = ref.get_state()
    ref.close()
    nrm = lambda a: float(np.abs(a).sum())
    return {"rho": nrm(U_mp[0] - U_64[0]) / nrm(U_64[0]),
            "m": nrm(U_mp[1:1 + dim] - U_64[1:1 + dim]) / nrm(U_64[1:1 + dim]),
            "E": nrm(U_mp[dim + 1] - U_64[dim + 1]) / nrm(U_64[dim + 1]),
            "steps": steps, "norm": "L1 relative",
            "positivity_violations": int(not (st.min_rho > 0 and st.min_eps > 0)),
            "fp64_redo_steps": st.fp64_redo,
            "min_rho": st.min_rho, "min_eps": st.min_eps,
            "reference": "the FP64 path of this library (parity-tested against the "
                         "oracle) from the same state with the same time steps"}


def single_mode(args):
    """One workload as the headline (profiling runs): --dim 3, --ns, --mixed
    or the default 2D FP64 workload with --only."""
    dim = 3 if args.ns else args.dim
    n = args.n or (4096 if dim == 2 else 256)
    mesh, U = workload(dim, n, args.seed)
    t0 = time.perf_counter()
    graph = abi.Graph(mesh)
    mixed = 2 if args.fp32_eval else int(args.mixed)
    res = run_steps(graph, U, dim, mixed, args.steps, args.warmup, ns=args.ns,
                    mu=args.mu, precond=args.precond)
    setup_s = time.perf_counter() - t0 - res["elapsed"]
    cb = copy_bandwidth(res["solver"])
    res["solver"].close()
    tag = (f"{dim}d_{n}" + ("_mixed" if mixed else "") + ("_fp32" if mixed == 2 else "")
           + ("_ns" if args.ns else ""))
    out = base_line("DoF-updates/s per SSP-RK stage", res["value"], args.steps,
                    args.warmup, res["ms_per_step"],
                    ("f64 (f32 storage, f32 graph-viscosity arithmetic)" if mixed == 2
                     else "f64 (f32 storage)" if mixed else "f64"),
                    {"workload": workload_name(dim, n, args.seed, bool(mixed), args.ns,
                                               args.mu, args.precond)
                     + (", FP32 evaluation of lambda_max, |c_ij| and the entropy indicator"
                        if mixed == 2 else ""),
                     "nodes": res["N"], "stages_per_step": 6 if args.ns else 3})
    s = summary(res, dim, tag)
    out["roofline"] = s.pop("roofline")
    out.update(s)
    out.update(cb)
    out["kernels"] = res["kernels"]
    out["setup_s"] = setup_s
    if args.ns:
        out["cg_iterations"] = {"velocity": [c[0] for c in res["cg"]],
                                "energy": [c[1] for c in res["cg"]],
                                "low_order": [c[2] for c in res["cg"]],
                                "limited_steps": sum(c[3] for c in res["cg"])}
    if mixed and not args.no_error:
        out["error_vs_fp64"] = mixed_error(graph, U, 50, dim, PRECISIONS[mixed])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(
            dim, args.cpu_sample or (1024 if dim == 2 else (64 if args.ns else 96)),
            args.seed, ns=args.ns, mu=args.mu, single=dim == 2 and not args.ns)
    return out


def full_run(args):
    """The headline 2D FP64 workload, then the other configurations."""
    def say(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    # C2: headline
    n2 = args.n or 4096
    mesh2, U2 = workload(2, n2, args.seed)
    t0 = time.perf_counter()
    g2 = abi.Graph(mesh2)
    res = run_steps(g2, U2, 2, False, args.steps, args.warmup)
    setup_s = time.perf_counter() - t0 - res["elapsed"]
    cb = copy_bandwidth(res["solver"])
    res["solver"].close()
    say(f"2D fp64 {res['ms_per_step']:.2f} ms/step")
    out = base_line("DoF-updates/s per SSP-RK stage", res["value"], args.steps, args.warmup,
                    res["ms_per_step"], "f64",
                    {"workload": workload_name(2, n2, args.seed), "nodes": res["N"],
                     "stages_per_step": 3})
    s = summary(res, 2, f"2d_{n2}")
    out["roofline"] = s.pop("roofline")
    out.update(s)
    out.update(cb)
    out["kernels"] = res["kernels"]
    out["setup_s"] = setup_s
    configs = {}

    # C4: the same workload in mixed precision; L1 difference after 50 steps
    res = run_steps(g2, U2, 2, True, args.steps, args.warmup)
    res["solver"].close()
    say(f"2D mixed {res['ms_per_step']:.2f} ms/step")
    configs["mixed_2d"] = summary(
        res, 2, f"2d_{n2}_mixed",
        {"workload": workload_name(2, n2, args.seed, mixed=True),
         "dtype": "f64 (f32 storage)", "speedup_vs_fp64": res["value"] / out["value"],
         "error_vs_fp64": mixed_error(g2, U2, 50, 2)})
    say("2D mixed error", configs["mixed_2d"]["error_vs_fp64"]["rho"])
    # C4 with FP32 evaluation of the graph-viscosity sweep
    res = run_steps(g2, U2, 2, 2, args.steps, args.warmup)
    res["solver"].close()
    say(f"2D mixed fp32-eval {res['ms_per_step']:.2f} ms/step")
    configs["mixed_fp32_2d"] = summary(
        res, 2, f"2d_{n2}_mixed_fp32",
        {"workload": workload_name(2, n2, args.seed, mixed=True) + ", FP32 evaluation of "
                     "lambda_max, |c_ij| and the entropy indicator",
         "dtype": "f64 (f32 storage, f32 graph-viscosity arithmetic)",
         "speedup_vs_fp64": res["value"] / out["value"],
         "speedup_vs_mixed": res["ms_per_step"] and
         configs["mixed_2d"]["ms_per_step"] / res["ms_per_step"],
         "error_vs_fp64": mixed_error(g2, U2, 50, 2, abi.PREC_MIXED_FP32)})
    say("2D mixed fp32-eval error", configs["mixed_fp32_2d"]["error_vs_fp64"]["rho"])
    del g2, U2

    # C3: 3D shock tube, hyperbolic step and Navier-Stokes Strang step
    n3 = 256
    mesh3, U3 = workload(3, n3, args.seed)
    g3 = abi.Graph(mesh3)
    res = run_steps(g3, U3, 3, False, args.steps3, 2)
    res["solver"].close()
    say(f"3D fp64 {res['ms_per_step']:.2f} ms/step")
    configs["euler_3d"] = summary(res, 3, f"3d_{n3}",
                                  {"workload": workload_name(3, n3, args.seed),
                                   "steps": args.steps3})
    res = run_steps(g3, U3, 3, False, args.steps_ns, 1, ns=True)
    res["solver"].close()
    say(f"3D NS {res['ms_per_step']:.2f} ms/step")
    configs["navier_stokes_3d"] = summary(
        res, 3, f"3d_{n3}_ns",
        {"workload": workload_name(3, n3, args.seed, ns=True), "steps": args.steps_ns,
         "stages_per_step": 6,
         "cg_iterations": {"velocity": [c[0] for c in res["cg"]],
                           "energy": [c[1] for c in res["cg"]],
                           "limited_steps": sum(c[3] for c in res["cg"])}})
    del g3, U3

    # C5: serving, FP64 and mixed precision (captured step graphs), and FP64
    # with every unit stepped by persistent launches (one per chunk)
    if not args.no_serve:
        for mixed in (False, True):
            r = serve_bench(args, mixed)
            say(f"serving {'mixed' if mixed else 'fp64'} p50 {r['latency_ms']['p50']:.0f} ms")
            configs["serving_mixed" if mixed else "serving_fp64"] = r
        pa = argparse.Namespace(**vars(args))
        pa.persistent_rows = max(args.pack_nodes, 1 << 20)
        r = serve_bench(pa, False)
        say(f"serving fp64 persistent p50 {r['latency_ms']['p50']:.0f} ms")
        configs["serving_fp64_persistent"] = r
    out["configs"] = configs
    if not args.no_cpu_baseline:
        say("oracle baseline")
        out["cpu_baseline"] = cpu_baseline(2, args.cpu_sample or 1024, args.seed)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--steps3", type=int, default=10,
                    help="full run: timed steps of the 3D hyperbolic workload")
    ap.add_argument("--steps-ns", type=int, default=5,
                    help="full run: timed Strang steps of the Navier-Stokes workload")
    ap.add_argument("--only", action="store_true",
                    help="the headline (or --dim/--ns/--mixed) workload alone")
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3),
                    help="with --only: 2 (four-quadrant data on 4096^2 nodes) or 3 "
                         "(Mach-3 shock tube on 256^3 nodes, hyperbolic step)")
    ap.add_argument("--n", type=int, default=0,
                    help="nodes per direction of the headline workload")
    ap.add_argument("--ns", action="store_true",
                    help="alone: Navier-Stokes Strang steps (mu = 1e-4, kappa = 1.4e-4, "
                         "cv = 1/(gamma-1), CG rtol 1e-10)")
    ap.add_argument("--mu", type=float, default=1e-4,
                    help="Navier-Stokes: shear viscosity (kappa = 1.4 mu)")
    ap.add_argument("--precond", choices=("jacobi", "gmg"), default="jacobi",
                    help="Navier-Stokes: preconditioner of the parabolic CG (gmg: "
                         "FP32 multigrid V-cycle, for the viscous-dominated regime)")
    ap.add_argument("--mixed", action="store_true",
                    help="alone: mixed precision (FP32 storage of alpha, d_ij, F^H and "
                         "the limiter coefficients)")
    ap.add_argument("--fp32-eval", action="store_true",
                    help="alone: mixed precision with FP32 evaluation of lambda_max, "
                         "|c_ij| and the entropy indicator")
    ap.add_argument("--serve", action="store_true",
                    help="alone: the serving workload (FP64, or mixed with --mixed)")
    ap.add_argument("--no-serve", action="store_true",
                    help="full run without the serving workload")
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
    ap.add_argument("--persistent-rows", type=int, default=0,
                    help="serving: units (solvers or packs) of at most this many rows "
                         "are stepped by one persistent launch per chunk; larger ones "
                         "by captured step graphs (0: none)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues for the serving streams (GPU_MAX_HW_QUEUES, "
                         "at most 32)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle sample, nodes per direction (default 1024 in "
                         "2D, 96 in 3D)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true",
                    help="alone, mixed precision: skip the 50-step comparison with the "
                         "FP64 path (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the hyperbolic step is benchmarked "
              "on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    # set before the first HIP call of the process; the serving streams are
    # spread over these hardware queues (the other workloads use one stream)
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(max(args.hw_queues, 1), 32))

    if args.serve:
        r = serve_bench(args, args.mixed)
        out = base_line("DoF-updates/s per SSP-RK stage; p50/p99 request latency",
                        r.pop("value"), args.serve_steps, 1, None, r.pop("dtype"),
                        {"workload": r.pop("workload"), "requests": r.pop("requests")})
        out.update(r)
    elif args.only or args.dim == 3 or args.ns or args.mixed or args.fp32_eval:
        out = single_mode(args)
    else:
        out = full_run(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
