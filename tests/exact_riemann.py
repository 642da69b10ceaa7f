"""Exact solution of the 1-D Riemann problem for a gamma-law gas.

Test-only.  The star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 with the
shock (Rankine-Hugoniot) and rarefaction (isentropic) branches of the
pressure function (Toro 2009, ch. 4); the solution is then sampled along
x/t.  It is an independent check of the hydro oracle: it shares nothing with
either the oracle or the GPU library.
"""
import math

import numpy as np


def _f_and_df(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    e = (g - 1.0) / (2.0 * g)
    f = 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0)
    df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g=1.4, tol=1e-14):
    """(p*, u*) of the Riemann problem by Newton iteration."""
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    # two-rarefaction guess
    e = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) /
         (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-12)
    for _ in range(100):
        fl, dfl = _f_and_df(p, rl, pl, cl, g)
        fr, dfr = _f_and_df(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, g)
    fr, _ = _f_and_df(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def waves(rl, ul, pl, rr, ur, pr, g=1.4):
    """Star state and wave speeds: dict with p, u, rho_l, rho_r and the speeds
    of the left and right waves (head/tail of rarefactions, shock speeds)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    out = {"p": ps, "u": us}
    if ps > pl:
        out["rho_l"] = rl * ((ps / pl + gm) / (gm * ps / pl + 1.0))
        out["left_shock"] = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
    else:
        out["rho_l"] = rl * (ps / pl) ** (1.0 / g)
        cls = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        out["left_head"] = ul - cl
        out["left_tail"] = us - cls
    if ps > pr:
        out["rho_r"] = rr * ((ps / pr + gm) / (gm * ps / pr + 1.0))
        out["right_shock"] = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
    else:
        out["rho_r"] = rr * (ps / pr) ** (1.0 / g)
        crs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
        out["right_head"] = ur + cr
        out["right_tail"] = us + crs
    return out


def sample(xi, rl, ul, pl, rr, ur, pr, g=1.4):
    """(rho, u, p) at similarity coordinates xi = (x - x0) / t (numpy array)."""
    xi = np.asarray(xi, dtype=np.float64)
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    r, v, q = rl, ul, pl
                else:
                    r, v, q = rl * ((ps / pl + gm) / (gm * ps / pl + 1.0)), us, ps
            else:
                shl = ul - cl
                stl = us - cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s <= shl:
                    r, v, q = rl, ul, pl
                elif s >= stl:
                    r, v, q = rl * (ps / pl) ** (1.0 / g), us, ps
                else:
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    v = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    r = rl * (c / cl) ** (2.0 / (g - 1))
                    q = pl * (c / cl) ** (2.0 * g / (g - 1))
        else:  # right of the contact
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    r, v, q = rr, ur, pr
                else:
                    r, v, q = rr * ((ps / pr + gm) / (gm * ps / pr + 1.0)), us, ps
            else:
                shr = ur + cr
                str_ = us + cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s >= shr:
                    r, v, q = rr, ur, pr
                elif s <= str_:
                    r, v, q = rr * (ps / pr) ** (1.0 / g), us, ps
                else:
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    v = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    r = rr * (c / cr) ** (2.0 / (g - 1))
                    q = pr * (c / cr) ** (2.0 * g / (g - 1))
        rho[idx], u[idx], p[idx] = r, v, q
    return rho, u, p


def cell_average(xc, dx, t, x0, left, right, g=1.4, nsub=64):
    """Cell averages of the exact density over cells centred at xc (midpoint
    rule on nsub sub-points per cell)."""
    off = (np.arange(nsub) + 0.5) / nsub - 0.5
    xs = xc[:, None] + off[None, :] * dx
    r, _, _ = sample((xs - x0) / t, *left, *right, g=g)
    return r.mean(axis=1)
