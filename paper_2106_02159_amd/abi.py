"""Thin ctypes binding of libns (include/ns.h): argument marshalling only.

Every computation runs in the HIP library; this module only converts NumPy
arrays and Python numbers to the C ABI.  Importing it does not touch the GPU.
``lib()`` raises ``ImportError`` when ``libns.so`` has not been built: there
is no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libns.so")

# status codes (ns.h)
NS_OK, NS_EINVAL, NS_ENOMEM, NS_EHIP = 0, -1, -2, -3
NS_ENOTADMISSIBLE, NS_ECFL, NS_EBOUNDS, NS_ESTATE, NS_ECG = -4, -5, -6, -7, -8
NS_EABORT = -9
FCT_AUTO, FCT_ALWAYS = 0, 1
PREC_FP64, PREC_MIXED, PREC_MIXED_FP32 = 0, 1, 2
IND_ENTROPY, IND_ONE, IND_ZERO = 0, 1, 2
LIM_CONVEX, LIM_LOW, LIM_HIGH = 0, 1, 2
ON_DEVICE, NO_PROJECT = 1, 2
DBG = {"stage_out": 0, "d": 1, "alpha": 2, "UL": 3, "FH": 4, "bounds": 5,
       "lt1": 6, "lt2": 7, "U1": 8, "roots": 9}

EXPORTED = [
    "ns_graph_create", "ns_graph_destroy", "ns_graph_info", "ns_graph_export",
    "ns_graph_stencil",
    "ns_solver_create", "ns_solver_destroy", "ns_set_state", "ns_get_state",
    "ns_compute_dt", "ns_step", "ns_step_cfl", "ns_fe_stage", "ns_get_debug",
    "ns_sync", "ns_stream", "ns_profile_enable", "ns_profile_count",
    "ns_profile_get", "ns_copy_bench", "ns_device_bytes", "ns_last_error",
    "ns_create_error",
    "ns_strerror", "ns_set_viscous", "ns_step_parabolic", "ns_step_strang",
    "ns_step_strang_cfl", "ns_parabolic_info", "ns_step_cfl_async", "ns_query",
    "ns_inflight",
    "ns_async_finish", "ns_solver_footprint", "ns_server_create", "ns_server_destroy",
    "ns_server_submit", "ns_server_progress", "ns_server_request", "ns_server_result",
    "ns_server_stats_get", "ns_server_error", "ns_pack_footprint", "ns_pack_create",
    "ns_pack_destroy", "ns_pack_set_state", "ns_pack_get_state", "ns_pack_step_cfl_async",
    "ns_pack_inflight", "ns_pack_finish", "ns_pack_error", "ns_set_boundary",
    "ns_step_adaptive", "ns_stats", "ns_stats_noalloc", "ns_step_cfl_persistent",
    "ns_cancel", "ns_pack_step_cfl_persistent", "ns_pack_cancel",
]


class NSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("periodic", C.c_int * 3)]


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double),
                ("indicator", C.c_int), ("limiter", C.c_int), ("passes", C.c_int),
                ("relax", C.c_double), ("precision", C.c_int)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run "
                              "`python -m paper_2106_02159_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        sig = {
            "ns_graph_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(vp)]),
            "ns_graph_destroy": (None, [vp]),
            "ns_graph_info": (C.c_int, [vp, i64p, i64p, C.POINTER(C.c_int),
                                        C.POINTER(C.c_int)]),
            "ns_graph_export": (C.c_int, [vp, vp, vp, vp, vp, vp]),
            "ns_graph_stencil": (C.c_int, [vp, C.c_int64, C.c_int64, vp, vp, vp]),
            "ns_solver_create": (C.c_int, [vp, C.POINTER(Params), vp, C.POINTER(vp)]),
            "ns_solver_destroy": (None, [vp]),
            "ns_set_state": (C.c_int, [vp, vp, C.c_int]),
            "ns_get_state": (C.c_int, [vp, vp, C.c_int]),
            "ns_compute_dt": (C.c_int, [vp, dp]),
            "ns_step": (C.c_int, [vp, C.c_double]),
            "ns_step_cfl": (C.c_int, [vp, dp]),
            "ns_fe_stage": (C.c_int, [vp, C.c_double]),
            "ns_get_debug": (C.c_int, [vp, C.c_int, vp]),
            "ns_sync": (C.c_int, [vp]),
            "ns_stream": (vp, [vp]),
            "ns_profile_enable": (C.c_int, [vp, C.c_int]),
            "ns_profile_count": (C.c_int, [vp]),
            "ns_profile_get": (C.c_int, [vp, C.c_int, C.POINTER(C.c_char_p), i64p, dp]),
            "ns_copy_bench": (C.c_int, [vp, C.c_int64, C.c_int, C.c_int, dp]),
            "ns_device_bytes": (C.c_int64, [vp]),
            "ns_last_error": (C.c_char_p, [vp]),
            "ns_create_error": (C.c_char_p, []),
            "ns_strerror": (C.c_char_p, [C.c_int]),
            "ns_set_viscous": (C.c_int, [vp, C.POINTER(Viscous)]),
            "ns_step_parabolic": (C.c_int, [vp, C.c_double]),
            "ns_step_strang": (C.c_int, [vp, C.c_double]),
            "ns_step_strang_cfl": (C.c_int, [vp, dp]),
            "ns_parabolic_info": (C.c_int, [vp, C.POINTER(ParInfo)]),
            "ns_stats": (C.c_int, [vp, C.POINTER(Stats)]),
            "ns_stats_noalloc": (C.c_int, [vp, C.POINTER(Stats)]),
            "ns_step_cfl_async": (C.c_int, [vp, C.c_int]),
            "ns_query": (C.c_int, [vp, C.POINTER(C.c_int)]),
            "ns_inflight": (C.c_int, [vp, C.POINTER(C.c_int)]),
            "ns_async_finish": (C.c_int, [vp, dp]),
            "ns_solver_footprint": (C.c_int, [vp, C.POINTER(Params), i64p]),
            "ns_server_create": (C.c_int, [C.POINTER(ServerParams), C.POINTER(vp)]),
            "ns_server_destroy": (None, [vp]),
            "ns_server_submit": (C.c_int, [vp, C.POINTER(MeshDesc), vp, C.c_int, i64p]),
            "ns_server_progress": (C.c_int, [vp, C.POINTER(C.c_int)]),
            "ns_server_request": (C.c_int, [vp, C.c_int64, C.POINTER(RequestInfo)]),
            "ns_server_result": (C.c_int, [vp, C.c_int64, vp]),
            "ns_server_stats_get": (C.c_int, [vp, C.POINTER(ServerStats)]),
            "ns_server_error": (C.c_char_p, [vp, C.c_int64]),
            "ns_pack_footprint": (C.c_int, [vp, C.c_int, C.POINTER(Params), i64p]),
            "ns_pack_create": (C.c_int, [vp, C.c_int, C.POINTER(Params), vp,
                                         C.POINTER(vp)]),
            "ns_pack_destroy": (None, [vp]),
            "ns_pack_set_state": (C.c_int, [vp, C.c_int, vp]),
            "ns_pack_get_state": (C.c_int, [vp, C.c_int, vp]),
            "ns_pack_step_cfl_async": (C.c_int, [vp, C.c_int]),
            "ns_pack_inflight": (C.c_int, [vp, C.POINTER(C.c_int)]),
            "ns_pack_finish": (C.c_int, [vp, C.POINTER(C.c_int), dp]),
            "ns_pack_error": (C.c_char_p, [vp]),
            "ns_set_boundary": (C.c_int, [vp, C.POINTER(Boundary)]),
            "ns_step_adaptive": (C.c_int, [vp, C.c_double, dp, dp]),
            "ns_step_cfl_persistent": (C.c_int, [vp, C.c_int, C.c_double]),
            "ns_cancel": (C.c_int, [vp]),
            "ns_pack_step_cfl_persistent": (C.c_int, [vp, C.c_int, C.c_double]),
            "ns_pack_cancel": (C.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data


def mesh_desc(mesh) -> MeshDesc:
    """From any object with dim, n, lo, hi, periodic (workloads.Mesh)."""
    d = MeshDesc()
    d.dim = mesh.dim
    for k in range(3):
        d.n[k] = int(mesh.n[k]) if k < mesh.dim else 1
        d.lo[k] = float(mesh.lo[k]) if k < mesh.dim else 0.0
        d.hi[k] = float(mesh.hi[k]) if k < mesh.dim else 1.0
        d.periodic[k] = int(bool(mesh.periodic[k])) if k < mesh.dim else 0
    return d


class Graph:
    """ns_graph_create / ns_graph_info / ns_graph_export."""

    def __init__(self, mesh):
        L = lib()
        h = C.c_void_p()
        desc = mesh_desc(mesh)
        rc = L.ns_graph_create(C.byref(desc), C.byref(h))
        if rc != NS_OK:
            raise NSError(rc, L.ns_create_error().decode())
        self.h = h
        N, nnz = C.c_int64(), C.c_int64()
        dim, W = C.c_int(), C.c_int()
        L.ns_graph_info(h, C.byref(N), C.byref(nnz), C.byref(dim), C.byref(W))
        self.N, self.nnz, self.dim, self.W = N.value, nnz.value, dim.value, W.value

    def export(self):
        N, W, dim = self.N, self.W, self.dim
        col = np.empty((W, N), np.int32)
        mij = np.empty((W, N))
        cij = np.empty((dim, W, N))
        mi = np.empty(N)
        bnd = np.empty((dim, N))
        lib().ns_graph_export(self.h, _ptr(col), _ptr(mij), _ptr(cij), _ptr(mi),
                              _ptr(bnd))
        return dict(col=col, mij=mij, cij=cij, mi=mi, bnd=bnd)

    def stencil(self, base=0, rows=None):
        """Stencil entries as the kernels derive them (ns_graph_stencil) for
        the mesh at row `base` plus padding rows: col (W, rows) int32, mij
        (W, rows), cij (dim, W, rows)."""
        rows = self.N if rows is None else rows
        col = np.empty((self.W, rows), np.int32)
        mij = np.empty((self.W, rows))
        cij = np.empty((self.dim, self.W, rows))
        rc = lib().ns_graph_stencil(self.h, base, rows, _ptr(col), _ptr(mij), _ptr(cij))
        if rc != NS_OK:
            raise NSError(rc, "ns_graph_stencil")
        return dict(col=col, mij=mij, cij=cij)

    def close(self):
        if getattr(self, "h", None):
            lib().ns_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Viscous(C.Structure):
    _fields_ = [("mu", C.c_double), ("lam", C.c_double), ("kappa", C.c_double),
                ("cv", C.c_double), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int),
                ("fct", C.c_int), ("precond", C.c_int)]


PC_JACOBI, PC_GMG = 0, 1


class ParInfo(C.Structure):
    _fields_ = [("it_v", C.c_int), ("it_e", C.c_int), ("it_l", C.c_int),
                ("fct", C.c_int), ("min_eH", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("min_rho", C.c_double), ("min_eps", C.c_double),
                ("argmin_rho", C.c_int64), ("argmin_eps", C.c_int64),
                ("edges", C.c_int64), ("limited1", C.c_int64), ("limited2", C.c_int64),
                ("roots1", C.c_int64), ("roots2", C.c_int64),
                ("cg_it_v", C.c_int), ("cg_it_e", C.c_int), ("cg_it_l", C.c_int),
                ("fct", C.c_int), ("min_eH", C.c_double), ("fp64_redo", C.c_int)]


class Boundary(C.Structure):
    _fields_ = [("kind", C.c_int * 6), ("method", C.c_int), ("state", (C.c_double * 5) * 6)]


BC_SLIP, BC_NONREFLECTING = 0, 1
NR_CHARACTERISTIC, NR_GODUNOV = 0, 1


class ServerParams(C.Structure):
    _fields_ = [("mem_bytes", C.c_int64), ("max_running", C.c_int), ("chunk", C.c_int),
                ("depth", C.c_int), ("solver", Params), ("pack_nodes", C.c_int64),
                ("pack_max", C.c_int), ("persistent_rows", C.c_int64)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int), ("status", C.c_int), ("steps", C.c_int),
                ("bytes", C.c_int64), ("n_nodes", C.c_int64), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_finish", C.c_double), ("t_sim", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "finished", "queued", "running",
                                        "peak_running", "peak_bytes", "bytes_in_use",
                                        "units")] + \
               [(k, C.c_double) for k in ("host_admit_s", "host_topup_s", "host_finish_s")]


REQ_QUEUED, REQ_RUNNING, REQ_FINISHED = 0, 1, 2


def footprint(graph, gamma=1.4, cfl=0.5, precision=PREC_FP64, **kw) -> int:
    """Device bytes a solver of these parameters would allocate."""
    prm = Params(gamma, cfl, kw.get("indicator", IND_ENTROPY), kw.get("limiter", LIM_CONVEX),
                 kw.get("passes", 2), kw.get("relax", 1.0), precision)
    b = C.c_int64()
    rc = lib().ns_solver_footprint(graph.h, C.byref(prm), C.byref(b))
    if rc != NS_OK:
        raise NSError(rc, "footprint")
    return b.value


def _params(gamma, cfl, precision, kw) -> Params:
    return Params(gamma, cfl, kw.get("indicator", IND_ENTROPY), kw.get("limiter", LIM_CONVEX),
                  kw.get("passes", 2), kw.get("relax", 1.0), precision)


def pack_footprint(graphs, gamma=1.4, cfl=0.5, precision=PREC_FP64, **kw) -> int:
    """Device bytes a pack of these graphs would allocate."""
    prm = _params(gamma, cfl, precision, kw)
    hs = (C.c_void_p * len(graphs))(*[g.h.value for g in graphs])
    b = C.c_int64()
    rc = lib().ns_pack_footprint(hs, len(graphs), C.byref(prm), C.byref(b))
    if rc != NS_OK:
        raise NSError(rc, "pack footprint")
    return b.value


class Pack:
    """ns_pack_*: several meshes advanced by the same kernel launches."""

    def __init__(self, graphs, gamma=1.4, cfl=0.5, precision=PREC_FP64, stream=None, **kw):
        L = lib()
        self.graphs = list(graphs)
        prm = _params(gamma, cfl, precision, kw)
        hs = (C.c_void_p * len(self.graphs))(*[g.h.value for g in self.graphs])
        h = C.c_void_p()
        rc = L.ns_pack_create(hs, len(self.graphs), C.byref(prm), stream, C.byref(h))
        if rc != NS_OK:
            raise NSError(rc, L.ns_create_error().decode())
        self.h = h

    def _check(self, rc):
        if rc != NS_OK:
            raise NSError(rc, lib().ns_pack_error(self.h).decode())
        return rc

    def set_state(self, r: int, U):
        U = np.ascontiguousarray(U, np.float64)
        g = self.graphs[r]
        assert U.shape == (g.dim + 2, g.N)
        self._check(lib().ns_pack_set_state(self.h, int(r), _ptr(U)))

    def get_state(self, r: int) -> np.ndarray:
        g = self.graphs[r]
        out = np.empty((g.dim + 2, g.N))
        self._check(lib().ns_pack_get_state(self.h, int(r), _ptr(out)))
        return out

    def step_cfl_async(self, nsteps: int):
        self._check(lib().ns_pack_step_cfl_async(self.h, int(nsteps)))

    def step_cfl_persistent(self, nsteps: int, wait_s: float = 10.0):
        self._check(lib().ns_pack_step_cfl_persistent(self.h, int(nsteps), float(wait_s)))

    def cancel(self):
        self._check(lib().ns_pack_cancel(self.h))

    def inflight(self) -> int:
        n = C.c_int()
        self._check(lib().ns_pack_inflight(self.h, C.byref(n)))
        return n.value

    def finish(self):
        """(status per member, time advanced per member)."""
        n = len(self.graphs)
        st = (C.c_int * n)()
        t = np.zeros(n)
        self._check(lib().ns_pack_finish(self.h, st, t.ctypes.data_as(C.POINTER(C.c_double))))
        return list(st), t

    def close(self):
        if getattr(self, "h", None):
            lib().ns_pack_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Server:
    """ns_server_*: continuous batching of independent simulations."""

    def __init__(self, mem_bytes, max_running=64, gamma=1.4, cfl=0.5,
                 precision=PREC_FP64, chunk=2, depth=2, pack_nodes=0, pack_max=64,
                 persistent_rows=0):
        L = lib()
        self.prm = ServerParams(int(mem_bytes), int(max_running), int(chunk), int(depth),
                                Params(gamma, cfl, IND_ENTROPY, LIM_CONVEX, 2, 1.0,
                                       precision), int(pack_nodes), int(pack_max),
                                int(persistent_rows))
        h = C.c_void_p()
        rc = L.ns_server_create(C.byref(self.prm), C.byref(h))
        if rc != NS_OK:
            raise NSError(rc, "server create")
        self.h = h
        self.meshes = {}

    def submit(self, mesh, U, steps: int) -> int:
        U = np.ascontiguousarray(U, np.float64)
        d = mesh_desc(mesh)
        rid = C.c_int64()
        rc = lib().ns_server_submit(self.h, C.byref(d), _ptr(U), int(steps), C.byref(rid))
        if rc != NS_OK:
            raise NSError(rc, lib().ns_server_error(self.h, 0).decode())
        self.meshes[rid.value] = (mesh.dim + 2, mesh.N)
        return rid.value

    def progress(self) -> int:
        n = C.c_int()
        rc = lib().ns_server_progress(self.h, C.byref(n))
        if rc != NS_OK:
            raise NSError(rc, "server progress")
        return n.value

    def request(self, rid: int) -> RequestInfo:
        info = RequestInfo()
        rc = lib().ns_server_request(self.h, int(rid), C.byref(info))
        if rc != NS_OK:
            raise NSError(rc, "unknown request")
        return info

    def result(self, rid: int):
        """(state, status) of a finished request; forgets the request."""
        nc, N = self.meshes.pop(rid)
        out = np.empty((nc, N))
        rc = lib().ns_server_result(self.h, int(rid), _ptr(out))
        return out, rc

    def error(self, rid: int) -> str:
        return lib().ns_server_error(self.h, int(rid)).decode()

    def stats(self) -> ServerStats:
        st = ServerStats()
        lib().ns_server_stats_get(self.h, C.byref(st))
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().ns_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """ns_solver_create and the per-solver calls."""

    def __init__(self, graph: Graph, gamma=1.4, cfl=0.5, indicator=IND_ENTROPY,
                 limiter=LIM_CONVEX, passes=2, relax=1.0, precision=PREC_FP64,
                 stream=None):
        L = lib()
        self.graph = graph  # keep alive
        self.prm = Params(gamma, cfl, indicator, limiter, passes, relax, precision)
        h = C.c_void_p()
        rc = L.ns_solver_create(graph.h, C.byref(self.prm),
                                C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != NS_OK:
            raise NSError(rc, L.ns_create_error().decode())
        self.h = h
        self.N, self.dim, self.W = graph.N, graph.dim, graph.W
        self.nc = self.dim + 2

    def _check(self, rc):
        if rc != NS_OK:
            raise NSError(rc, lib().ns_last_error(self.h).decode())
        return rc

    def set_state(self, U, project=True):
        U = np.ascontiguousarray(U, np.float64)
        assert U.shape == (self.nc, self.N)
        self._check(lib().ns_set_state(self.h, _ptr(U), 0 if project else NO_PROJECT))

    def get_state(self):
        out = np.empty((self.nc, self.N))
        self._check(lib().ns_get_state(self.h, _ptr(out), 0))
        return out

    def set_state_device(self, ptr: int, project=True):
        """State from a component-major nc*N FP64 array in device memory at
        address ptr (complete before the call)."""
        self._check(lib().ns_set_state(self.h, C.c_void_p(ptr),
                                       ON_DEVICE | (0 if project else NO_PROJECT)))

    def get_state_device(self, ptr: int):
        """State into a component-major nc*N FP64 array in device memory at
        address ptr (complete on return)."""
        self._check(lib().ns_get_state(self.h, C.c_void_p(ptr), ON_DEVICE))

    def compute_dt(self) -> float:
        dt = C.c_double()
        self._check(lib().ns_compute_dt(self.h, C.byref(dt)))
        return dt.value

    def step(self, dt: float):
        return self._check(lib().ns_step(self.h, float(dt)))

    def step_cfl(self) -> float:
        dt = C.c_double()
        self._check(lib().ns_step_cfl(self.h, C.byref(dt)))
        return dt.value

    def step_status(self, dt: float) -> int:
        """ns_step returning the raw status instead of raising."""
        return lib().ns_step(self.h, float(dt))

    # -- parabolic sub-step and Strang composition --------------------------
    def set_viscous(self, mu=1e-4, lam=0.0, kappa=1.4e-4, cv=2.5, cg_rtol=1e-10,
                    cg_maxit=500, fct=FCT_AUTO, precond=PC_JACOBI):
        self.vprm = Viscous(mu, lam, kappa, cv, cg_rtol, cg_maxit, fct, precond)
        self._check(lib().ns_set_viscous(self.h, C.byref(self.vprm)))

    def step_parabolic(self, dt: float):
        return self._check(lib().ns_step_parabolic(self.h, float(dt)))

    def step_parabolic_status(self, dt: float) -> int:
        return lib().ns_step_parabolic(self.h, float(dt))

    def step_strang(self, tau: float):
        return self._check(lib().ns_step_strang(self.h, float(tau)))

    def step_strang_cfl(self) -> float:
        tau = C.c_double()
        self._check(lib().ns_step_strang_cfl(self.h, C.byref(tau)))
        return tau.value

    def parabolic_info(self) -> ParInfo:
        info = ParInfo()
        self._check(lib().ns_parabolic_info(self.h, C.byref(info)))
        return info

    def stats(self) -> Stats:
        out = Stats()
        self._check(lib().ns_stats(self.h, C.byref(out)))
        return out

    def stats_noalloc(self) -> Stats:
        out = Stats()
        self._check(lib().ns_stats_noalloc(self.h, C.byref(out)))
        return out

    # -- asynchronous stepping ---------------------------------------------
    def step_cfl_async(self, nsteps: int):
        return self._check(lib().ns_step_cfl_async(self.h, int(nsteps)))

    def step_cfl_persistent(self, nsteps: int, wait_s: float = 10.0):
        """nsteps CFL steps as one persistent launch (asynchronous)."""
        return self._check(lib().ns_step_cfl_persistent(self.h, int(nsteps), float(wait_s)))

    def cancel(self):
        return self._check(lib().ns_cancel(self.h))

    def step_adaptive(self, c_start: float):
        """(dt, c) of one step with the adaptive CFL number."""
        dt, c = C.c_double(), C.c_double()
        self._check(lib().ns_step_adaptive(self.h, float(c_start), C.byref(dt), C.byref(c)))
        return dt.value, c.value

    def set_boundary(self, kind, method=NR_CHARACTERISTIC, state=None):
        """Faces f = 2*dir + side: kind[f] in BC_*; state[f] the far-field
        conserved state (rho, m, E) of a non-reflecting face."""
        b = Boundary()
        for f in range(6):
            b.kind[f] = int(kind[f]) if f < len(kind) else BC_SLIP
            if state is not None and f < len(state) and state[f] is not None:
                for c, v in enumerate(state[f]):
                    b.state[f][c] = float(v)
        b.method = int(method)
        self._check(lib().ns_set_boundary(self.h, C.byref(b)))

    def query(self) -> bool:
        done = C.c_int()
        self._check(lib().ns_query(self.h, C.byref(done)))
        return bool(done.value)

    def async_finish(self):
        """(status, time advanced) of the steps enqueued since the last call."""
        t = C.c_double()
        rc = lib().ns_async_finish(self.h, C.byref(t))
        return rc, t.value

    def fe_stage(self, dt: float) -> int:
        return lib().ns_fe_stage(self.h, float(dt))

    def debug(self, what: str):
        N, W, nc = self.N, self.W, self.nc
        shape = {"stage_out": (nc, N), "d": (W, N), "alpha": (N,), "UL": (nc, N),
                 "FH": (nc, N), "bounds": (3, N), "lt1": (W, N), "lt2": (W, N),
                 "U1": (nc, N), "roots": (2,)}[what]
        out = np.empty(shape)
        self._check(lib().ns_get_debug(self.h, DBG[what], _ptr(out)))
        return out

    def sync(self):
        self._check(lib().ns_sync(self.h))

    def stream(self) -> int:
        return lib().ns_stream(self.h) or 0

    def profile(self, on: bool):
        self._check(lib().ns_profile_enable(self.h, 1 if on else 0))

    def profile_report(self):
        L = lib()
        out = {}
        for k in range(L.ns_profile_count(self.h)):
            name = C.c_char_p()
            n = C.c_int64()
            ms = C.c_double()
            self._check(L.ns_profile_get(self.h, k, C.byref(name), C.byref(n),
                                         C.byref(ms)))
            out[name.value.decode()] = (n.value, ms.value)
        return out

    def copy_bench(self, nbytes: int, reps: int = 10, word: int = 16) -> float:
        """Average time (ms) of a plain device copy of nbytes moving `word`
        (8 or 16) bytes per lane."""
        ms = C.c_double()
        self._check(lib().ns_copy_bench(self.h, int(nbytes), int(reps), int(word),
                                        C.byref(ms)))
        return ms.value

    def device_bytes(self) -> int:
        return lib().ns_device_bytes(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().ns_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
