"""Exact solution of the 1D Riemann problem for the gamma-law Euler equations.

TEST INFRASTRUCTURE ONLY.  Textbook construction (E. F. Toro, *Riemann
Solvers and Numerical Methods for Fluid Dynamics*, 3rd ed., ch. 4): the star
pressure p* is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, found here by
safeguarded Newton iteration to round-off; the self-similar solution is then
sampled at x/t.  Used to pin the oracle's wave-speed bound (it must dominate
the exact extreme wave speeds) and to measure convergence on 1D Riemann
problems.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, ak, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        f = (p - pk) * q
        df = q * (1.0 - 0.5 * (p - pk) / (p + B))
    else:  # rarefaction
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * ak / (g - 1.0) * ((p / pk) ** e - 1.0)
        df = 1.0 / (rho * ak) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g=1.4):
    """Return (p*, u*) of the exact Riemann solution (no vacuum)."""
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    if 2.0 / (g - 1.0) * (al + ar) <= ur - ul:
        raise ValueError("vacuum is generated")
    du = ur - ul
    # bracket: f is increasing in p; f(0) < 0
    lo, hi = 0.0, max(pl, pr)
    while _fk(hi, rl, pl, al, g)[0] + _fk(hi, rr, pr, ar, g)[0] + du < 0.0:
        hi *= 2.0
    e = (g - 1.0) / (2.0 * g)
    p = ((al + ar - 0.5 * (g - 1.0) * du) /
         (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    p = min(max(p, 1e-300), hi)
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, al, g)
        fr, dfr = _fk(p, rr, pr, ar, g)
        f = fl + fr + du
        if f > 0.0:
            hi = p
        else:
            lo = p
        pn = p - f / (dfl + dfr)
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= 1e-15 * max(p, pn):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, al, g)
    fr, _ = _fk(p, rr, pr, ar, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def extreme_wave_speeds(rl, ul, pl, rr, ur, pr, g=1.4):
    """(lambda_1^-, lambda_3^+): leftmost and rightmost wave speeds."""
    ps, _ = star_state(rl, ul, pl, rr, ur, pr, g)
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    c = (g + 1.0) / (2.0 * g)
    l1 = ul - al * math.sqrt(1.0 + c * max(ps / pl - 1.0, 0.0))
    l3 = ur + ar * math.sqrt(1.0 + c * max(ps / pr - 1.0, 0.0))
    return l1, l3, ps


def max_wave_speed(rl, ul, pl, rr, ur, pr, g=1.4):
    l1, l3, _ = extreme_wave_speeds(rl, ul, pl, rr, ur, pr, g)
    return max(-l1, l3, 0.0)


def sample(rl, ul, pl, rr, ur, pr, xi, g=1.4):
    """Density, velocity, pressure at similarity coordinates xi = x/t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    xi = np.atleast_1d(np.asarray(xi, np.float64))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for k, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    rho[k], u[k], p[k] = rl, ul, pl
                else:
                    rho[k] = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                    u[k], p[k] = us, ps
            else:  # left rarefaction
                shl = ul - al
                asl = al * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - asl
                if s <= shl:
                    rho[k], u[k], p[k] = rl, ul, pl
                elif s >= stl:
                    rho[k] = rl * (ps / pl) ** (1.0 / g)
                    u[k], p[k] = us, ps
                else:
                    c = 2.0 / (g + 1) + (g - 1) / ((g + 1) * al) * (ul - s)
                    rho[k] = rl * c ** (2.0 / (g - 1))
                    u[k] = 2.0 / (g + 1) * (al + (g - 1) / 2 * ul + s)
                    p[k] = pl * c ** (2 * g / (g - 1))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    rho[k], u[k], p[k] = rr, ur, pr
                else:
                    rho[k] = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                    u[k], p[k] = us, ps
            else:  # right rarefaction
                shr = ur + ar
                asr = ar * (ps / pr) ** ((g - 1) / (2 * g))
                stR = us + asr
                if s >= shr:
                    rho[k], u[k], p[k] = rr, ur, pr
                elif s <= stR:
                    rho[k] = rr * (ps / pr) ** (1.0 / g)
                    u[k], p[k] = us, ps
                else:
                    c = 2.0 / (g + 1) - (g - 1) / ((g + 1) * ar) * (ur - s)
                    rho[k] = rr * c ** (2.0 / (g - 1))
                    u[k] = 2.0 / (g + 1) * (-ar + (g - 1) / 2 * ur + s)
                    p[k] = pr * c ** (2 * g / (g - 1))
    return rho, u, p
