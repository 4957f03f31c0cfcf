"""Exact solution of the one-dimensional Riemann problem of an ideal gas
(test infrastructure: the analytic reference of the shock-tube run, not a
step of the pair passes).

Two uniform states (rho, u, P) meet at x0 at t = 0. The star-region
pressure p* solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where each f_K is the
velocity jump across a shock (p > P_K, Rankine-Hugoniot) or a rarefaction
(p <= P_K, isentropic); p* is found by Newton iteration from the
two-rarefaction estimate, u* = (u_L + u_R + f_R - f_L) / 2, and the profile
at x follows from the similarity variable xi = (x - x0) / t: left wave,
contact at u*, right wave. This is the standard exact solver of gas
dynamics textbooks, written out here in our own code.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, P, gamma):
    """Velocity change across the wave joining (rho, P) to pressure p, and its
    derivative in p."""
    c = math.sqrt(gamma * P / rho)
    if p > P:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * P
        q = math.sqrt(A / (p + B))
        return (p - P) * q, q * (1.0 - 0.5 * (p - P) / (p + B))
    e = (gamma - 1.0) / (2.0 * gamma)
    r = p / P
    return 2.0 * c / (gamma - 1.0) * (r ** e - 1.0), r ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * c)


def star(left, right, gamma):
    """(p*, u*) of the Riemann problem between left = (rho, u, P) and right."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    e = (gamma - 1.0) / (2.0 * gamma)
    # two-rarefaction estimate as the starting point
    num = cl + cr - 0.5 * (gamma - 1.0) * (ur - ul)
    p = max((num / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e), 1e-12)
    for _ in range(100):
        fl, dl = _f(p, rl, pl, gamma)
        fr, dr = _f(p, rr, pr, gamma)
        step = (fl + fr + ur - ul) / (dl + dr)
        pn = max(p - step, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, gamma)
    fr, _ = _f(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur + fr - fl)


def sample(x, t, x0, left, right, gamma):
    """(rho, u, P) arrays of the exact solution at positions x, time t > 0."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star(left, right, gamma)
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1, g2 = (gamma - 1.0) / (gamma + 1.0), 2.0 / (gamma + 1.0)
    xi = (np.asarray(x, dtype=np.float64) - x0) / t
    rho, u, P = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    for k, s in enumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                r_star = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                sh = ul - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl
                                         + (gamma - 1.0) / (2.0 * gamma))
                st = (rl, ul, pl) if s < sh else (r_star, us, ps)
            else:  # left rarefaction
                r_star = rl * (ps / pl) ** (1.0 / gamma)
                c_star = cl * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                head, tail = ul - cl, us - c_star
                if s < head:
                    st = (rl, ul, pl)
                elif s > tail:
                    st = (r_star, us, ps)
                else:
                    uf = g2 * (cl + 0.5 * (gamma - 1.0) * ul + s)
                    cf = g2 * (cl + 0.5 * (gamma - 1.0) * (ul - s))
                    rf = rl * (cf / cl) ** (2.0 / (gamma - 1.0))
                    st = (rf, uf, pl * (cf / cl) ** (2.0 * gamma / (gamma - 1.0)))
        else:  # right of the contact
            if ps > pr:  # right shock
                r_star = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                sh = ur + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr
                                         + (gamma - 1.0) / (2.0 * gamma))
                st = (rr, ur, pr) if s > sh else (r_star, us, ps)
            else:  # right rarefaction
                r_star = rr * (ps / pr) ** (1.0 / gamma)
                c_star = cr * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                head, tail = ur + cr, us + c_star
                if s > head:
                    st = (rr, ur, pr)
                elif s < tail:
                    st = (r_star, us, ps)
                else:
                    uf = g2 * (-cr + 0.5 * (gamma - 1.0) * ur + s)
                    cf = g2 * (cr - 0.5 * (gamma - 1.0) * (ur - s))
                    rf = rr * (cf / cr) ** (2.0 / (gamma - 1.0))
                    st = (rf, uf, pr * (cf / cr) ** (2.0 * gamma / (gamma - 1.0)))
        rho[k], u[k], P[k] = st
    return rho, u, P
