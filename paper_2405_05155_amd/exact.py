"""Exact solution of the 1-D Riemann problem of an ideal gas, the reference
the shock-tube checks compare against (evaluation only: nothing in the
library calls it).

The star pressure solves f_l(p) + f_r(p) + (u_r - u_l) = 0 with the shock
(Rankine-Hugoniot) branch for p above a side's pressure and the isentropic
rarefaction branch below, by bisection; the density is then sampled from the
wave pattern (shock or rarefaction fan on each side of the contact) at
xi = x / t.
"""
import math


def riemann_density(rl, ul, pl, rr, ur, pr, xi, gamma=1.4):
    """Density of the exact solution of the 1-D Riemann problem of an ideal
    gas at x/t = xi: the star pressure from the shock (Rankine-Hugoniot) and
    rarefaction (isentropic) branches by bisection, then the wave pattern
    sampled at xi (textbook construction)."""
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1, g2 = (gamma - 1.0) / (2.0 * gamma), (gamma + 1.0) / (2.0 * gamma)

    def branch(p, rk, pk, ck):
        if p > pk:
            a, b = 2.0 / ((gamma + 1.0) * rk), (gamma - 1.0) / (gamma + 1.0) * pk
            return (p - pk) * math.sqrt(a / (p + b))
        return 2.0 * ck / (gamma - 1.0) * ((p / pk) ** g1 - 1.0)

    lo, hi = 1e-12, 100.0 * max(pl, pr)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if branch(mid, rl, pl, cl) + branch(mid, rr, pr, cr) + (ur - ul) > 0.0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (branch(ps, rr, pr, cr) - branch(ps, rl, pl, cl))
    q = (gamma - 1.0) / (gamma + 1.0)
    if xi <= us:  # left of the contact
        if ps > pl:
            s = ul - cl * math.sqrt(g2 * ps / pl + g1)
            return rl if xi < s else rl * (ps / pl + q) / (q * ps / pl + 1.0)
        head, tail = ul - cl, us - cl * (ps / pl) ** g1
        if xi < head:
            return rl
        if xi > tail:
            return rl * (ps / pl) ** (1.0 / gamma)
        return rl * (2.0 / (gamma + 1.0) + (gamma - 1.0) / ((gamma + 1.0) * cl) * (ul - xi)) ** (2.0 / (gamma - 1.0))
    if ps > pr:
        s = ur + cr * math.sqrt(g2 * ps / pr + g1)
        return rr if xi > s else rr * (ps / pr + q) / (q * ps / pr + 1.0)
    head, tail = ur + cr, us + cr * (ps / pr) ** g1
    if xi > head:
        return rr
    if xi < tail:
        return rr * (ps / pr) ** (1.0 / gamma)
    return rr * (2.0 / (gamma + 1.0) - (gamma - 1.0) / ((gamma + 1.0) * cr) * (ur - xi)) ** (2.0 / (gamma - 1.0))


def sod_density(xi, gamma=1.4):
    """Sod's problem: (rho, u, p) = (1, 0, 1) left, (0.125, 0, 0.1) right."""
    return riemann_density(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, xi, gamma)
