"""Exact solution of the Riemann problem for the 1-D Euler equations of an
ideal gas (textbook two-shock/two-rarefaction construction with a Newton
iteration on the star pressure).  Used to pin the oracle's shock-tube runs."""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, ck, gamma):
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    pr = p / pk
    f = 2.0 * ck / (gamma - 1.0) * (pr ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = 1.0 / (rho * ck) * pr ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma):
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _f(p, rl, pl, cl, gamma)
        fr, dfr = _f(p, rr, pr, cr, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-14 * p:
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, gamma)
    fr, _ = _f(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, gamma, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0) / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    g = gamma
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for j, s in enumerate(xi.ravel()):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                st = (rl, ul, pl) if s <= sl else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1 / g)
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                sh, stl = ul - cl, us - cs
                if s <= sh:
                    st = (rl, ul, pl)
                elif s >= stl:
                    st = (rs, us, ps)
                else:
                    uu = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    cc = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rr_ = rl * (cc / cl) ** (2 / (g - 1))
                    st = (rr_, uu, pl * (cc / cl) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                rs = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                st = (rr, ur, pr) if s >= sr else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1 / g)
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                sh, stl = ur + cr, us + cs
                if s >= sh:
                    st = (rr, ur, pr)
                elif s <= stl:
                    st = (rs, us, ps)
                else:
                    uu = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    cc = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    rr_ = rr * (cc / cr) ** (2 / (g - 1))
                    st = (rr_, uu, pr * (cc / cr) ** (2 * g / (g - 1)))
        rho.ravel()[j], u.ravel()[j], p.ravel()[j] = st
    return rho, u, p


def wave_speeds(left, right, gamma):
    """(rarefaction head, contact, shock) speeds for a left-rarefaction /
    right-shock problem such as Sod."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    g = gamma
    sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
    return ul - cl, us, sr
