"""Exact solution of the 1D Euler Riemann problem for an ideal gas (the
classical two-rarefaction/two-shock pressure function with Newton iteration on
the star pressure), written from the Rankine-Hugoniot and isentropic relations.
Used only to pin the oracle's shock-tube runs (Sec. 4.2)."""
import math

import numpy as np


def _pressure_function(p, rho, u, pk, g):
    c = math.sqrt(g * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * c / (g - 1.0) * (r - 1.0), 1.0 / (rho * c) * (p / pk) ** (-(g + 1.0) / (2.0 * g))


def star_state(left, right, g):
    rl, ul, pl = left
    rr, ur, pr = right
    p = max(1e-10, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _pressure_function(p, rl, ul, pl, g)
        fr, dr = _pressure_function(p, rr, ur, pr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_function(p, rl, ul, pl, g)
    fr, _ = _pressure_function(p, rr, ur, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, g, xi):
    """Primitive (rho, u, p) at similarity coordinate xi = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = np.zeros((3, len(xi)))
    for n, s in enumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    out[:, n] = (rl, ul, pl)
                else:
                    rs = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                    out[:, n] = (rs, us, ps)
            else:
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s <= ul - cl:
                    out[:, n] = (rl, ul, pl)
                elif s >= us - csl:
                    out[:, n] = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    rho = rl * (c / cl) ** (2 / (g - 1))
                    out[:, n] = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    out[:, n] = (rr, ur, pr)
                else:
                    rs = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                    out[:, n] = (rs, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s >= ur + cr:
                    out[:, n] = (rr, ur, pr)
                elif s <= us + csr:
                    out[:, n] = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    rho = rr * (c / cr) ** (2 / (g - 1))
                    out[:, n] = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out


def cell_average_density(left, right, g, x0, t, edges, nsub=40):
    xs = []
    for a, b in zip(edges[:-1], edges[1:]):
        xs.append(a + (np.arange(nsub) + 0.5) / nsub * (b - a))
    xs = np.concatenate(xs)
    rho = sample(left, right, g, (xs - x0) / t)[0]
    return rho.reshape(-1, nsub).mean(axis=1)
