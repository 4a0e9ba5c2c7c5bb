"""Python handle on the plain C oracle (``ns_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product package.

``build()`` compiles ``libns_oracle.so`` with gcc (``-O2``, no fast-math, no
FMA contraction).  ``Graph`` wraps the oracle's quadrature-assembled graph and
exposes the stage, step and time-step routines on NumPy arrays in the same
structure-of-arrays layout the library uses: ``U[c, i]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "ns_oracle.c"), os.path.join(HERE, "ns_oracle_parabolic.c"),
        os.path.join(HERE, "ns_oracle_bc.c")]
LIB = os.path.join(HERE, "libns_oracle.so")

IND_ENTROPY, IND_ONE, IND_ZERO = 0, 1, 2
LIM_CONVEX, LIM_LOW, LIM_HIGH = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle shared library (plain C, gcc)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
               "-fno-fast-math", "-Wall", "-o", LIB] + SRCS + ["-lm"]
        subprocess.check_call(cmd)
    return LIB


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double),
                ("indicator", C.c_int), ("limiter", C.c_int),
                ("passes", C.c_int), ("relax", C.c_double),
                ("volume", C.c_double)]


class _Visc(C.Structure):
    _fields_ = [("mu", C.c_double), ("lam", C.c_double), ("kappa", C.c_double),
                ("cv", C.c_double), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int),
                ("fct", C.c_int)]


class ParInfo(C.Structure):
    _fields_ = [("it_v", C.c_int), ("it_e", C.c_int), ("it_l", C.c_int),
                ("fct", C.c_int), ("min_eH", C.c_double), ("min_e", C.c_double)]


class _Boundary(C.Structure):
    _fields_ = [("kind", C.c_int * 6), ("method", C.c_int),
                ("state", (C.c_double * 5) * 6)]


BC_SLIP, BC_NONREFLECTING = 0, 1
NR_CHARACTERISTIC, NR_GODUNOV = 0, 1


def boundary(kind, method=NR_CHARACTERISTIC, state=None) -> _Boundary:
    """Faces f = 2*dir + side (low, high end): kind[f] in BC_*; state[f] the
    far-field conserved state (rho, m, E) of a non-reflecting face."""
    b = _Boundary()
    for f in range(6):
        b.kind[f] = int(kind[f]) if f < len(kind) else BC_SLIP
        if state is not None and f < len(state) and state[f] is not None:
            for c, v in enumerate(state[f]):
                b.state[f][c] = float(v)
    b.method = int(method)
    return b


class _Debug(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("d", "alpha", "UL", "FH", "bounds", "lt1", "l1", "lt2", "l2",
                 "U1")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        lp = C.POINTER(C.c_long)
        L.orc_graph_build.argtypes = [C.c_int, lp, dp, dp, C.POINTER(C.c_int),
                                      C.POINTER(C.c_void_p)]
        L.orc_graph_free.argtypes = [C.c_void_p]
        L.orc_graph_N.argtypes = [C.c_void_p]
        L.orc_graph_N.restype = C.c_long
        L.orc_graph_nnz.argtypes = [C.c_void_p]
        L.orc_graph_nnz.restype = C.c_long
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_graph_export.argtypes = [C.c_void_p] + [C.c_void_p] * 9
        L.orc_pressure.argtypes = [C.c_double, C.c_int, dp]
        L.orc_pressure.restype = C.c_double
        L.orc_lambda_max.argtypes = [C.c_double, C.c_int, dp, dp, dp]
        L.orc_lambda_max.restype = C.c_double
        L.orc_line_search.argtypes = [C.c_double, C.c_int, dp, dp, C.c_double,
                                      C.c_double, C.c_double]
        L.orc_line_search.restype = C.c_double
        L.orc_compute_dt.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp]
        L.orc_fe_stage.argtypes = [C.c_void_p, C.POINTER(_Params), dp,
                                   C.c_double, dp, C.POINTER(_Debug)]
        L.orc_slip_bc.argtypes = [C.c_void_p, dp]
        L.orc_ssprk3_step.argtypes = [C.c_void_p, C.POINTER(_Params), dp,
                                      C.c_double, dp]
        L.orc_high_order_direct.argtypes = [C.c_void_p, C.POINTER(_Params), dp,
                                            C.c_double, dp]
        vpp = C.POINTER(_Visc)
        for name in ("orc_stress_apply", "orc_heat_apply", "orc_dissipation"):
            getattr(L, name).argtypes = [C.c_void_p, vpp, dp, dp]
        L.orc_heat_matrix.argtypes = [C.c_void_p, vpp, dp]
        L.orc_parabolic_step.argtypes = [C.c_void_p, vpp, dp, C.c_double, dp,
                                         C.POINTER(ParInfo)]
        L.orc_strang_step.argtypes = [C.c_void_p, C.POINTER(_Params), vpp, dp,
                                      C.c_double, dp, C.POINTER(ParInfo)]
        L.orc_riemann_star.argtypes = [C.c_double] * 7 + [dp, dp]
        L.orc_riemann_sample.argtypes = [C.c_double] * 8 + [dp, dp, dp,
                                                            C.POINTER(C.c_int)]
        L.orc_nr_state.argtypes = [C.c_double, C.c_int, C.c_int, dp, dp, dp, dp]
        L.orc_boundary_bc.argtypes = [C.c_void_p, C.POINTER(_Params),
                                      C.POINTER(_Boundary), dp]
        L.orc_ssprk3_step_bc.argtypes = [C.c_void_p, C.POINTER(_Params),
                                         C.POINTER(_Boundary), dp, C.c_double, dp]
        L.orc_ssprk3_step_adaptive.argtypes = [C.c_void_p, C.POINTER(_Params),
                                               C.POINTER(_Boundary), dp, C.c_double,
                                               dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads used by the oracle's parallel row loops from now on."""
    lib().orc_set_num_threads(int(n))


def params(gamma=1.4, cfl=0.5, indicator=IND_ENTROPY, limiter=LIM_CONVEX,
           passes=2, relax=1.0, volume=0.0) -> _Params:
    """volume: |Omega| entering the bound relaxation; 0 = the mesh's own
    (sum of m_i).  A sub-mesh window cut from a larger domain passes that
    domain's volume so that its rows see the same relaxed bounds."""
    return _Params(gamma, cfl, indicator, limiter, passes, relax, volume)


def visc(mu=1e-4, lam=0.0, kappa=1.4e-4, cv=2.5, cg_rtol=1e-10, cg_maxit=500,
         fct=0) -> _Visc:
    """Viscous data of the parabolic step (stress coefficients mu, lambda,
    heat coefficient kappa / cv), the CG tolerance and the limiting mode
    (0: only when the high-order internal energy is not positive, 1: always)."""
    return _Visc(mu, lam, kappa, cv, cg_rtol, cg_maxit, fct)


def lambda_max(gamma, ui, uj, n) -> float:
    ui = np.ascontiguousarray(ui, np.float64)
    uj = np.ascontiguousarray(uj, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    return lib().orc_lambda_max(gamma, len(n), _dp(ui), _dp(uj), _dp(n))


def line_search(gamma, u, P, rho_min, rho_max, phi_min) -> float:
    u = np.ascontiguousarray(u, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    return lib().orc_line_search(gamma, len(u) - 2, _dp(u), _dp(P), rho_min,
                                 rho_max, phi_min)


def riemann_star(gamma, left, right):
    """(p*, u*) of the 1D Riemann problem with primitive data (rho, u, p)
    left and right, or None for vacuum."""
    ps, us = C.c_double(), C.c_double()
    rc = lib().orc_riemann_star(gamma, *map(float, left), *map(float, right),
                                C.byref(ps), C.byref(us))
    return None if rc else (ps.value, us.value)


def riemann_sample(gamma, left, right, xi=0.0):
    """(rho, u, p, side) of the Riemann solution at x/t = xi (side -1 / +1:
    left / right of the contact), or None for vacuum."""
    r, u, p, sd = C.c_double(), C.c_double(), C.c_double(), C.c_int()
    rc = lib().orc_riemann_sample(gamma, *map(float, left), *map(float, right), float(xi),
                                  C.byref(r), C.byref(u), C.byref(p), C.byref(sd))
    return None if rc else (r.value, u.value, p.value, sd.value)


def nr_state(gamma, method, U, UD, n):
    """(post-processed state, admissible) of one non-reflecting node."""
    U = np.ascontiguousarray(U, np.float64)
    UD = np.ascontiguousarray(UD, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    out = np.empty_like(U)
    rc = lib().orc_nr_state(gamma, len(n), int(method), _dp(U), _dp(UD), _dp(n), _dp(out))
    return out, rc == 0


def pressure(gamma, u) -> float:
    u = np.ascontiguousarray(u, np.float64)
    return lib().orc_pressure(gamma, len(u) - 2, _dp(u))


class Graph:
    """Oracle graph of a uniform Q1 mesh on a box (Gauss-quadrature assembly)."""

    def __init__(self, dim, n, lo, hi, periodic, export=True):
        L = lib()
        self.dim = dim
        nn = (C.c_long * 3)(*(list(n) + [1] * (3 - len(n))))
        lo3 = (C.c_double * 3)(*(list(lo) + [0.0] * (3 - len(lo))))
        hi3 = (C.c_double * 3)(*(list(hi) + [0.0] * (3 - len(hi))))
        pp = (C.c_int * 3)(*([int(bool(x)) for x in periodic] +
                             [0] * (3 - len(periodic))))
        h = C.c_void_p()
        rc = L.orc_graph_build(dim, nn, lo3, hi3, pp, C.byref(h))
        if rc != 0:
            raise ValueError("oracle graph build failed")
        self.h = h
        self.N = L.orc_graph_N(h)
        self.nnz = L.orc_graph_nnz(h)
        self.nc = dim + 2
        if export:  # numpy copies of the graph (tests of the graph itself)
            self._export()

    def _export(self):
        N, nnz, dim = self.N, self.nnz, self.dim
        self.row_ptr = np.empty(N + 1, np.int64)
        self.col = np.empty(nnz, np.int64)
        self.tr = np.empty(nnz, np.int64)
        self.mij = np.empty(nnz, np.float64)
        self.cij = np.empty((dim, nnz), np.float64)
        self.bpair = np.empty((dim, nnz), np.float64)
        self.mi = np.empty(N, np.float64)
        self.bnd = np.empty((dim, N), np.float64)
        self.on_wall = np.empty(N, np.int32)
        lib().orc_graph_export(self.h, *[a.ctypes.data for a in (
            self.row_ptr, self.col, self.tr, self.mij, self.cij, self.bpair,
            self.mi, self.bnd, self.on_wall)])

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_graph_free(self.h)
                self.h = None
        except Exception:
            pass

    def compute_dt(self, prm, U) -> float:
        U = np.ascontiguousarray(U, np.float64)
        tau = C.c_double()
        lib().orc_compute_dt(self.h, C.byref(prm), _dp(U), C.byref(tau))
        return tau.value

    def fe_stage(self, prm, U, tau, debug=False):
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty_like(U)
        if not debug:
            st = lib().orc_fe_stage(self.h, C.byref(prm), _dp(U), tau, _dp(out),
                                    None)
            return out, st
        N, nnz, nc = self.N, self.nnz, self.nc
        dbg = {"d": np.zeros(nnz), "alpha": np.zeros(N),
               "UL": np.zeros((nc, N)), "FH": np.zeros((nc, N)),
               "bounds": np.zeros((3, N)), "lt1": np.zeros(nnz),
               "l1": np.zeros(nnz), "lt2": np.zeros(nnz), "l2": np.zeros(nnz),
               "U1": np.zeros((nc, N))}
        D = _Debug(*[dbg[k].ctypes.data for k in
                     ("d", "alpha", "UL", "FH", "bounds", "lt1", "l1", "lt2",
                      "l2", "U1")])
        st = lib().orc_fe_stage(self.h, C.byref(prm), _dp(U), tau, _dp(out),
                                C.byref(D))
        return out, st, dbg

    def slip_bc(self, U):
        U = np.array(U, np.float64, order="C", copy=True)
        lib().orc_slip_bc(self.h, _dp(U))
        return U

    def ssprk3_step(self, prm, U, tau, bnd=None):
        """One SSPRK(3,3) step; with `bnd` (oracle.boundary) the
        slip / non-reflecting post-processing after every stage, and the
        status has bit 1 set if a post-processed state was inadmissible."""
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty_like(U)
        if bnd is None:
            st = lib().orc_ssprk3_step(self.h, C.byref(prm), _dp(U), tau, _dp(out))
        else:
            st = lib().orc_ssprk3_step_bc(self.h, C.byref(prm), C.byref(bnd), _dp(U), tau,
                                          _dp(out))
        return out, st

    def ssprk3_step_adaptive(self, prm, U, c_start, bnd=None):
        """(U^{n+1}, tau, c) of a step with the adaptive CFL number (restart
        with c halved while a low-order state or a stage result is not
        admissible), or None if no c works."""
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty_like(U)
        tau, c = C.c_double(), C.c_double()
        rc = lib().orc_ssprk3_step_adaptive(self.h, C.byref(prm),
                                            C.byref(bnd) if bnd is not None else None,
                                            _dp(U), float(c_start), C.byref(tau),
                                            C.byref(c), _dp(out))
        return None if rc else (out, tau.value, c.value)

    def boundary_bc(self, prm, bnd, U):
        """(post-processed copy of U, status) with oracle.boundary `bnd`."""
        U = np.array(U, np.float64, order="C", copy=True)
        st = lib().orc_boundary_bc(self.h, C.byref(prm), C.byref(bnd), _dp(U))
        return U, st

    def high_order_direct(self, prm, U, tau):
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty_like(U)
        lib().orc_high_order_direct(self.h, C.byref(prm), _dp(U), tau, _dp(out))
        return out

    # -- parabolic sub-step ------------------------------------------------
    def stress_apply(self, vp, V):
        V = np.ascontiguousarray(V, np.float64)
        Y = np.empty_like(V)
        lib().orc_stress_apply(self.h, C.byref(vp), _dp(V), _dp(Y))
        return Y

    def heat_apply(self, vp, e):
        e = np.ascontiguousarray(e, np.float64)
        Y = np.empty_like(e)
        lib().orc_heat_apply(self.h, C.byref(vp), _dp(e), _dp(Y))
        return Y

    def heat_matrix(self, vp):
        B = np.empty(self.nnz)
        lib().orc_heat_matrix(self.h, C.byref(vp), _dp(B))
        return B

    def dissipation(self, vp, V):
        V = np.ascontiguousarray(V, np.float64)
        K = np.empty(self.N)
        lib().orc_dissipation(self.h, C.byref(vp), _dp(V), _dp(K))
        return K

    def parabolic_step(self, vp, U, dt):
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty_like(U)
        info = ParInfo()
        st = lib().orc_parabolic_step(self.h, C.byref(vp), _dp(U), dt, _dp(out),
                                      C.byref(info))
        return out, st, info

    def strang_step(self, prm, vp, U, tau):
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty_like(U)
        info = ParInfo()
        st = lib().orc_strang_step(self.h, C.byref(prm), C.byref(vp), _dp(U), tau,
                                   _dp(out), C.byref(info))
        return out, st, info

    # -- helpers for tests -------------------------------------------------
    def rows(self):
        for i in range(self.N):
            yield i, range(self.row_ptr[i], self.row_ptr[i + 1])
