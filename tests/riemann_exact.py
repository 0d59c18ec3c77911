"""Exact solution of the 1D Riemann problem for an ideal gas.

Textbook construction (two-rarefaction / two-shock pressure function with a
Newton iteration for the star pressure, then self-similar sampling), written
for the tests only: it gives the exact density of the shock tubes of the
paper's 1D Riemann table so the oracle's Euler path can be checked against
something that is not itself.
"""
import math

import numpy as np


def _f_and_df(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * ck / (g - 1.0) * (r - 1.0), (1.0 / (rho * ck)) * (p / pk) ** (-(g + 1.0) / (2.0 * g))


def star_state(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dfl = _f_and_df(p, rl, pl, cl, g)
        fr, dfr = _f_and_df(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, g)
    fr, _ = _f_and_df(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, xs, t, x0=0.0, g=1.4):
    """Exact (rho, u, p) at positions xs and time t > 0."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    out = np.zeros((3, len(xs)))
    gm = (g - 1.0) / (g + 1.0)
    for i, x in enumerate(xs):
        s = (x - x0) / t
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * ((ps / pl + gm) / (gm * ps / pl + 1.0))
                sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                out[:, i] = (rl, ul, pl) if s < sl else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                sh, st = ul - cl, us - cs
                if s < sh:
                    out[:, i] = (rl, ul, pl)
                elif s > st:
                    out[:, i] = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (g - 1.0))
                    out[:, i] = (r, u, pl * (c / cl) ** (2.0 * g / (g - 1.0)))
        else:
            if ps > pr:  # right shock
                rs = rr * ((ps / pr + gm) / (gm * ps / pr + 1.0))
                sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                out[:, i] = (rr, ur, pr) if s > sr else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1.0 / g)
                cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                sh, st = ur + cr, us + cs
                if s > sh:
                    out[:, i] = (rr, ur, pr)
                elif s < st:
                    out[:, i] = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
                    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
                    r = rr * (c / cr) ** (2.0 / (g - 1.0))
                    out[:, i] = (r, u, pr * (c / cr) ** (2.0 * g / (g - 1.0)))
    return out
