"""Exact solution of the Riemann problem of the 1-D Euler equations (ideal gas).

Textbook construction (two-shock/two-rarefaction star-state iteration on the
pressure function, then sampling of the self-similar solution).  Used only as
an independent pin of the oracle in its B = 0 limit.
"""
import math

import numpy as np


def _f(p, rho, pk, c, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    lo, hi = 1e-12, 10.0 * max(pl, pr)
    fun = lambda p: _f(p, rl, pl, cl, g) + _f(p, rr, pr, cr, g) + ur - ul
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fun(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_f(ps, rr, pr, cr, g) - _f(ps, rl, pl, cl, g))
    return ps, us


def sample(x, t, x0, left, right, g):
    """rho, u, p at positions x (array) and time t for an interface at x0."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = np.zeros((3, len(x)))
    for n, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:
            if ps > pl:  # left shock
                rs = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                out[:, n] = (rl, ul, pl) if s < sl else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                css = cl * (ps / pl) ** ((g - 1) / (2 * g))
                sh, st = ul - cl, us - css
                if s < sh:
                    out[:, n] = (rl, ul, pl)
                elif s > st:
                    out[:, n] = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (g - 1))
                    out[:, n] = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:  # right shock
                rs = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                out[:, n] = (rr, ur, pr) if s > sr else (rs, us, ps)
            else:  # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / g)
                css = cr * (ps / pr) ** ((g - 1) / (2 * g))
                sh, st = ur + cr, us + css
                if s > sh:
                    out[:, n] = (rr, ur, pr)
                elif s < st:
                    out[:, n] = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2.0 / (g - 1))
                    out[:, n] = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out
