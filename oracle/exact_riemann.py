"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations.

TEST INFRASTRUCTURE ONLY.  The paper checks its Sod shock-tube run against
the exact solution computed by the standard procedure of Toro's textbook
(Sec. 4.1, Sod).  This is that textbook procedure written out: the star
pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock
(Rankine-Hugoniot) branch for p > p_K and the rarefaction (isentropic) branch
otherwise; the solution is then sampled along rays x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho, pk, ck, gamma):
    if p > pk:  # shock branch
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction branch
    r = p / pk
    e = (gamma - 1.0) / (2.0 * gamma)
    f = 2.0 * ck / (gamma - 1.0) * (r ** e - 1.0)
    df = 1.0 / (rho * ck) * r ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma=1.4, tol=1e-14, max_iter=200):
    """Star-region pressure and velocity for left/right states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    du = ur - ul
    if 2.0 * (cl + cr) / (gamma - 1.0) <= du:
        raise ValueError("vacuum is generated; not supported")
    p = max(tol, 0.5 * (pl + pr) - 0.125 * du * (rl + rr) * (cl + cr))  # PVRS guess
    for _ in range(max_iter):
        fl, dfl = _f_and_df(p, rl, pl, cl, gamma)
        fr, dfr = _f_and_df(p, rr, pr, cr, gamma)
        pn = p - (fl + fr + du) / (dfl + dfr)
        if pn < tol:
            pn = tol
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, gamma)
    fr, _ = _f_and_df(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, xi, gamma=1.4):
    """Density, velocity and pressure at similarity coordinates xi = (x-x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for j, s in enumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    rho[j], u[j], p[j] = rl, ul, pl
                else:
                    rho[j] = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                    u[j], p[j] = us, ps
            else:  # left rarefaction
                shl = ul - cl
                cml = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                stl = us - cml
                if s <= shl:
                    rho[j], u[j], p[j] = rl, ul, pl
                elif s >= stl:
                    rho[j] = rl * (ps / pl) ** (1.0 / gamma)
                    u[j], p[j] = us, ps
                else:
                    c = 2.0 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - s))
                    u[j] = 2.0 / (gamma + 1) * (cl + (gamma - 1) / 2 * ul + s)
                    rho[j] = rl * (c / cl) ** (2.0 / (gamma - 1))
                    p[j] = pl * (c / cl) ** (2.0 * gamma / (gamma - 1))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    rho[j], u[j], p[j] = rr, ur, pr
                else:
                    rho[j] = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                    u[j], p[j] = us, ps
            else:  # right rarefaction
                shr = ur + cr
                cmr = cr * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                str_ = us + cmr
                if s >= shr:
                    rho[j], u[j], p[j] = rr, ur, pr
                elif s <= str_:
                    rho[j] = rr * (ps / pr) ** (1.0 / gamma)
                    u[j], p[j] = us, ps
                else:
                    c = 2.0 / (gamma + 1) * (cr - (gamma - 1) / 2 * (ur - s))
                    u[j] = 2.0 / (gamma + 1) * (-cr + (gamma - 1) / 2 * ur + s)
                    rho[j] = rr * (c / cr) ** (2.0 / (gamma - 1))
                    p[j] = pr * (c / cr) ** (2.0 * gamma / (gamma - 1))
    return rho, u, p


def wave_positions(left, right, t, x0=0.5, gamma=1.4):
    """Head and tail of the left rarefaction, contact and right shock at t
    (for the Sod configuration: left rarefaction, right shock)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    cml = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
    sr = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
    return dict(head=x0 + (ul - cl) * t, tail=x0 + (us - cml) * t,
                contact=x0 + us * t, shock=x0 + sr * t)
