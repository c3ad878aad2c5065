"""Exact solution of the Riemann problem for the 1D Euler equations with an
ideal-gas law (the textbook iterative solver: pressure function, Newton
iteration for the star pressure, self-similar sampling), used to pin the
oracle's shock tubes.  Independent of the oracle and of the GPU path."""
import math

import numpy as np


def _f_and_df(p, rk, pk, g):
    ck = math.sqrt(g * pk / rk)
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rk)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    e = (g - 1.0) / (2.0 * g)
    return (2.0 * ck / (g - 1.0)) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rk * ck)


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    # two-rarefaction guess, always positive
    e = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-14)
    for _ in range(200):
        fl, dl = _f_and_df(p, rl, pl, g)
        fr, dr = _f_and_df(p, rr, pr, g)
        f = fl + fr + (ur - ul)
        pn = max(p - f / (dl + dr), 1e-3 * p)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, g)
    fr, _ = _f_and_df(p, rr, pr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(rl, ul, pl, rr, ur, pr, g, xi):
    """(rho, u, p) at the similarity coordinates xi = (x - x0) / t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros((3,) + xi.shape)
    gm, gp = g - 1.0, g + 1.0
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            r, u, p, c = rl, ul, pl, math.sqrt(g * pl / rl)
            if ps > p:
                rs = r * ((ps / p + gm / gp) / (gm / gp * ps / p + 1.0))
                S = u - c * math.sqrt(gp / (2 * g) * ps / p + gm / (2 * g))
                val = (r, u, p) if s <= S else (rs, us, ps)
            else:
                rs = r * (ps / p) ** (1.0 / g)
                cs = c * (ps / p) ** (gm / (2 * g))
                if s <= u - c:
                    val = (r, u, p)
                elif s >= us - cs:
                    val = (rs, us, ps)
                else:
                    rf = r * (2.0 / gp + gm / (gp * c) * (u - s)) ** (2.0 / gm)
                    uf = 2.0 / gp * (c + gm / 2.0 * u + s)
                    pf = p * (2.0 / gp + gm / (gp * c) * (u - s)) ** (2.0 * g / gm)
                    val = (rf, uf, pf)
        else:  # right of contact
            r, u, p, c = rr, ur, pr, math.sqrt(g * pr / rr)
            if ps > p:
                rs = r * ((ps / p + gm / gp) / (gm / gp * ps / p + 1.0))
                S = u + c * math.sqrt(gp / (2 * g) * ps / p + gm / (2 * g))
                val = (r, u, p) if s >= S else (rs, us, ps)
            else:
                rs = r * (ps / p) ** (1.0 / g)
                cs = c * (ps / p) ** (gm / (2 * g))
                if s >= u + c:
                    val = (r, u, p)
                elif s <= us + cs:
                    val = (rs, us, ps)
                else:
                    rf = r * (2.0 / gp - gm / (gp * c) * (u - s)) ** (2.0 / gm)
                    uf = 2.0 / gp * (-c + gm / 2.0 * u + s)
                    pf = p * (2.0 / gp - gm / (gp * c) * (u - s)) ** (2.0 * g / gm)
                    val = (rf, uf, pf)
        out[(slice(None),) + idx] = val
    return out
