"""Pins of the exact Riemann solution used as the shock tube's analytic
reference, checked against the conservation laws and invariants it must
satisfy (not against its own formulas):

* across the shock, the speed from the mass flux also conserves momentum
  and energy (Rankine-Hugoniot), and the sampled jump sits at that speed;
* across the rarefaction fan the Riemann invariant u + 2c/(gamma-1) and
  the entropy P / rho^gamma are constant;
* pressure and velocity are continuous across the contact, density is not;
* equal states give a uniform solution; a symmetric collision stops the
  gas (u* = 0) with equal shocks on both sides.
"""
import math

import numpy as np
import pytest

from oracle import riemann

G = 5.0 / 3.0
SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.125))   # the shock tube's states (rho, u, P)


def _state(x, t=0.15, x0=0.5, left=SOD[0], right=SOD[1]):
    r, u, p = riemann.sample(np.atleast_1d(x), t, x0, left, right, G)
    return r[0], u[0], p[0]


def test_shock_satisfies_rankine_hugoniot():
    ps, us = riemann.star(*SOD, G)
    t, x0 = 0.15, 0.5
    xs = np.linspace(x0 + us * t + 1e-6, 1.0, 20001)
    r, u, p = riemann.sample(xs, t, x0, *SOD, G)
    k = int(np.argmax(r < 0.5 * (r[0] + SOD[1][0])))     # first pre-shock point
    r2, u2, p2 = r[k - 1], u[k - 1], p[k - 1]
    r1, u1, p1 = SOD[1]
    S = (r2 * u2 - r1 * u1) / (r2 - r1)
    mom = lambda r_, u_, p_: r_ * (u_ - S) ** 2 + p_
    ene = lambda r_, u_, p_: 0.5 * (u_ - S) ** 2 + G / (G - 1.0) * p_ / r_
    assert abs(mom(r2, u2, p2) - mom(r1, u1, p1)) < 1e-12 * mom(r1, u1, p1)
    assert abs(ene(r2, u2, p2) - ene(r1, u1, p1)) < 1e-12 * ene(r1, u1, p1)
    # the sampled jump sits at x0 + S t
    assert abs(xs[k] - (x0 + S * t)) <= 2 * (xs[1] - xs[0])
    assert p2 == pytest.approx(ps, rel=1e-14) and u2 == pytest.approx(us, rel=1e-14)


def test_rarefaction_invariants():
    ps, us = riemann.star(*SOD, G)
    rl, ul, pl = SOD[0]
    cl = math.sqrt(G * pl / rl)
    c_star = cl * (ps / pl) ** ((G - 1.0) / (2.0 * G))
    t, x0 = 0.15, 0.5
    xs = x0 + t * np.linspace(ul - cl, us - c_star, 41)
    r, u, p = riemann.sample(xs, t, x0, *SOD, G)
    c = np.sqrt(G * p / r)
    J = u + 2.0 * c / (G - 1.0)
    assert np.abs(J - (ul + 2.0 * cl / (G - 1.0))).max() < 1e-12
    s = p / r ** G
    assert np.abs(s / (pl / rl ** G) - 1.0).max() < 1e-12
    # the fan's edges join the left state and the star state
    assert r[0] == pytest.approx(rl, rel=1e-12) and p[-1] == pytest.approx(ps, rel=1e-10)


def test_contact_carries_only_a_density_jump():
    ps, us = riemann.star(*SOD, G)
    t, x0 = 0.15, 0.5
    xc = x0 + us * t
    a = _state(xc - 1e-9)
    b = _state(xc + 1e-9)
    assert a[1] == pytest.approx(b[1], rel=1e-14) and a[2] == pytest.approx(b[2], rel=1e-14)
    assert a[0] > b[0] * 1.2


def test_uniform_and_symmetric_cases():
    st = (0.7, 0.3, 2.0)
    r, u, p = riemann.sample(np.linspace(0, 1, 11), 0.1, 0.5, st, st, G)
    assert np.allclose(r, 0.7, rtol=1e-12) and np.allclose(u, 0.3, rtol=1e-12)
    assert np.allclose(p, 2.0, rtol=1e-12)
    ps, us = riemann.star((1.0, 1.0, 1.0), (1.0, -1.0, 1.0), G)
    assert abs(us) < 1e-14 and ps > 1.0
    r, u, p = riemann.sample(np.array([0.45, 0.55]), 0.05, 0.5, (1.0, 1.0, 1.0), (1.0, -1.0, 1.0), G)
    assert r[0] == pytest.approx(r[1], rel=1e-14) and u[0] == pytest.approx(-u[1], abs=1e-14)
