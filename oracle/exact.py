"""Exact solutions used to pin the oracle (test infrastructure).

* Sod shock tube: the exact Riemann solution of the Euler equations for an
  ideal gas (two-rarefaction/shock wave curves, Newton iteration on the star
  pressure), following the classical construction in E. F. Toro, "Riemann
  Solvers and Numerical Methods for Fluid Dynamics", Chapter 4.
* Isentropic vortex: the steady vortex of the Euler equations carried by a
  uniform stream; its exact solution at time t is the initial field translated
  by the stream velocity.
"""
from __future__ import annotations

import math

import numpy as np


def _wave_curve(p, rho_k, p_k, c_k, g):
    """f_k(p) and its derivative for the wave that connects state k to pressure p."""
    if p > p_k:  # shock
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        q = math.sqrt(A / (p + B))
        return (p - p_k) * q, q * (1.0 - 0.5 * (p - p_k) / (B + p))
    # rarefaction
    r = p / p_k
    f = 2.0 * c_k / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho_k * c_k) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(left, right, g=1.4, tol=1e-14):
    """Star pressure and velocity for primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(tol, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _wave_curve(p, rl, pl, cl, g)
        fr, dfr = _wave_curve(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p_new = max(tol, p - dp)
        if abs(p_new - p) <= tol * 0.5 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _wave_curve(p, rl, pl, cl, g)
    fr, _ = _wave_curve(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(left, right, xi, g=1.4):
    """Exact solution (rho, u, p) at similarity coordinates xi = x/t (arrays)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = riemann_star(left, right, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for n, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                SL = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                if s <= SL:
                    rho[n], u[n], p[n] = rl, ul, pl
                else:
                    rho[n] = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                    u[n], p[n] = us, ps
            else:  # left rarefaction
                cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                head, tail = ul - cl, us - cs
                if s <= head:
                    rho[n], u[n], p[n] = rl, ul, pl
                elif s >= tail:
                    rho[n] = rl * (ps / pl) ** (1.0 / g)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    u[n] = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    rho[n] = rl * (c / cl) ** (2.0 / (g - 1.0))
                    p[n] = pl * (c / cl) ** (2.0 * g / (g - 1.0))
        else:  # right of the contact
            if ps > pr:  # right shock
                SR = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                if s >= SR:
                    rho[n], u[n], p[n] = rr, ur, pr
                else:
                    rho[n] = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                    u[n], p[n] = us, ps
            else:  # right rarefaction
                cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                head, tail = ur + cr, us + cs
                if s >= head:
                    rho[n], u[n], p[n] = rr, ur, pr
                elif s <= tail:
                    rho[n] = rr * (ps / pr) ** (1.0 / g)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
                    u[n] = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
                    rho[n] = rr * (c / cr) ** (2.0 / (g - 1.0))
                    p[n] = pr * (c / cr) ** (2.0 * g / (g - 1.0))
    return rho, u, p


def sod_two_tube(x, t, g=1.4):
    """Density, velocity, pressure of the periodic two-tube Sod box of the
    workloads module: high state (1, 0, 1) on 0.5 < x < 1.5 of [0, 2), low
    state (0.125, 0, 0.1) elsewhere.  Valid while the waves of the two
    discontinuities do not meet (t <= 0.2)."""
    hi = (1.0, 0.0, 1.0)
    lo = (0.125, 0.0, 0.1)
    x = np.asarray(x, dtype=np.float64)
    # Right discontinuity at 1.5: high state on its left.
    rho_r, u_r, p_r = riemann_sample(hi, lo, (x - 1.5) / t, g)
    # Left discontinuity at 0.5: mirror image (low | high).
    rho_l, u_l, p_l = riemann_sample(lo, hi, (x - 0.5) / t, g)
    use_left = x < 1.0
    rho = np.where(use_left, rho_l, rho_r)
    u = np.where(use_left, u_l, u_r)
    p = np.where(use_left, p_l, p_r)
    return rho, u, p


def isentropic_vortex(x, y, t, L=20.0, strength=5.0, Ma=0.5, g=1.4, center=(10.0, 10.0), advect=(1.0, 1.0)):
    """Exact (rho, u, v, p) of the translating isentropic vortex.

    Around a centre moving with the stream, the tangential velocity is
    (strength / 2 pi) r exp((1 - r^2)/2); radial equilibrium of an isentropic
    gas then fixes p/rho = 1/(g Ma^2) - (g-1) strength^2 / (8 g pi^2) exp(1 - r^2)
    and rho = ((p/rho) / (p/rho)_inf)^(1/(g-1)), with rho_inf = 1."""
    dx = np.asarray(x) - center[0] - advect[0] * t
    dy = np.asarray(y) - center[1] - advect[1] * t
    dx = dx - L * np.round(dx / L)
    dy = dy - L * np.round(dy / L)
    r2 = dx * dx + dy * dy
    amp = strength / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    th_inf = 1.0 / (g * Ma * Ma)
    th = th_inf - (g - 1.0) * strength ** 2 / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
    rho = (th / th_inf) ** (1.0 / (g - 1.0))
    return rho, advect[0] - amp * dy, advect[1] + amp * dx, rho * th
