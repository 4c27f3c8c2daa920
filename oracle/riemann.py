"""Exact solution of the 1D Riemann problem of the Euler equations for an ideal
gas -- TEST INFRASTRUCTURE ONLY (a textbook pin for the oracle, not part of
the method).

Written from the standard construction (e.g. Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", ch. 4): the star pressure solves
f_L(p) + f_R(p) + u_R - u_L = 0 with the shock (Rankine-Hugoniot) or
rarefaction (isentropic) branch of f_K, and the self-similar solution is
sampled at xi = x / t.  The paper compares its shock tubes with this solution
(Sec. V.A-B).
"""
import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * np.sqrt(A / (p + B))
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, gamma=1.4):
    """Star-region pressure and velocity by bisection on the monotone
    pressure function (robust, no derivative needed)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum generated")

    def F(p):
        return _f(p, rl, pl, cl, g) + _f(p, rr, pr, cr, g) + ur - ul

    lo, hi = 1e-14, max(pl, pr)
    while F(hi) < 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if F(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_f(ps, rr, pr, cr, g) - _f(ps, rl, pl, cl, g))
    return ps, us


def sample(left, right, xi, gamma=1.4):
    """(rho, u, p) at the similarity coordinates xi (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((3, np.size(xi)))
    for k, s in enumerate(np.atleast_1d(xi)):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                SL = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= SL:
                    w = (rl, ul, pl)
                else:
                    w = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:  # left rarefaction
                SH = ul - cl
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                ST = us - cs
                if s <= SH:
                    w = (rl, ul, pl)
                elif s >= ST:
                    w = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    w = (rl * (c / cl) ** (2 / (g - 1)), u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:  # right of the contact
            if ps > pr:  # right shock
                SR = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= SR:
                    w = (rr, ur, pr)
                else:
                    w = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:  # right rarefaction
                SH = ur + cr
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                ST = us + cs
                if s >= SH:
                    w = (rr, ur, pr)
                elif s <= ST:
                    w = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    w = (rr * (c / cr) ** (2 / (g - 1)), u, pr * (c / cr) ** (2 * g / (g - 1)))
        out[:, k] = w
    return out


def wave_speeds(left, right, gamma=1.4):
    """Leftmost and rightmost signal speeds of the exact solution."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    if ps > pl:
        smin = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
    else:
        smin = ul - cl
    if ps > pr:
        smax = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
    else:
        smax = ur + cr
    return smin, smax
