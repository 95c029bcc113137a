"""Exact solution of the 1D Euler Riemann problem for an ideal gas.

Written from the standard pressure-function method (E.F. Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", ch. 4): the star pressure
is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, solved by Newton iteration,
then the self-similar solution is sampled at x/t.  Used only to pin the
oracle on two-state problems.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho, pk, ck, g):
    """Pressure function of one side and its derivative."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        f = (p - pk) * s
        df = s * (1.0 - 0.5 * (p - pk) / (p + B))
    else:  # rarefaction
        r = p / pk
        f = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g=1.4):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    # two-rarefaction initial guess
    z = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(100):
        fl, dfl = _f_and_df(p, rl, pl, cl, g)
        fr, dfr = _f_and_df(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, g)
    fr, _ = _f_and_df(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def star_densities(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    p, u = star_state(left, right, g)

    def side(rho, pk):
        if p > pk:
            r = p / pk
            q = (g - 1.0) / (g + 1.0)
            return rho * (r + q) / (q * r + 1.0)
        return rho * (p / pk) ** (1.0 / g)

    return side(rl, pl), side(rr, pr)


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) arrays at similarity coordinates xi = (x-x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    rsl, rsr = star_densities(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for i, s in enumerate(xi.flat):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                st = (rl, ul, pl) if s <= sl else (rsl, us, ps)
            else:
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                sh, stl = ul - cl, us - csl
                if s <= sh:
                    st = (rl, ul, pl)
                elif s >= stl:
                    st = (rsl, us, ps)
                else:
                    uu = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    cc = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rr_ = rl * (cc / cl) ** (2 / (g - 1))
                    st = (rr_, uu, pl * (cc / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                st = (rr, ur, pr) if s >= sr else (rsr, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                sh, stl = ur + cr, us + csr
                if s >= sh:
                    st = (rr, ur, pr)
                elif s <= stl:
                    st = (rsr, us, ps)
                else:
                    uu = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    cc = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    rr_ = rr * (cc / cr) ** (2 / (g - 1))
                    st = (rr_, uu, pr * (cc / cr) ** (2 * g / (g - 1)))
        rho.flat[i], u.flat[i], p.flat[i] = st
    return rho, u, p
