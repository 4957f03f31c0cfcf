"""Pins of the oracle's momentum and energy derivatives (eqs. mom, eng) with the
limited artificial viscosity (eqs. visc, mu, hatvi, phi, phiVL, rij, phiad).

What fixes them, independently of the oracle's own code:
  * Newton's third law (Sec. 2.2): the pair momentum terms cancel, so
    sum_i m_i dp_i/dt = 0;
  * eqs. (mom) and (eng) together conserve energy exactly: summing the pair
    terms, sum_i m_i du_i/dt + sum_i v_i . m_i dv_i/dt = 0 for any P, Q, v;
  * with A = 1, B = 0 and no viscosity the force reduces to the textbook
    volume-weighted SPH pressure force, checked here with a finite-difference
    kernel gradient;
  * for a linear flow the projected velocity difference vanishes and the
    viscosity switches off (Sec. 2.2); a sign error in the projection or the
    limiter turns it on;
  * v = 0 gives du/dt = 0 exactly, and a uniform state on a perfect lattice
    feels no force;
  * the limiter's closed-form values.
"""
import math

import numpy as np
import pytest

import crk_inputs as ci


def _run(orc, ps, prm, periodic=True, corr_override=None, gv_override=None):
    goff, gidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, periodic, 0)
    soff, sidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, periodic, 1)
    _, V, _ = orc.volume(ps.x, ps.y, ps.z, ps.H, goff, gidx, ps.L, periodic)
    mom = orc.moments(ps.x, ps.y, ps.z, ps.H, V, goff, gidx, ps.L, periodic)
    corr = corr_override or orc.corrections(mom)
    gv = gv_override if gv_override is not None else orc.gradv(
        ps.x, ps.y, ps.z, ps.H, ps.v, V, corr, goff, gidx, ps.L, periodic)
    dv, du, SF, SE = orc.derivatives(ps.x, ps.y, ps.z, ps.H, ps.v, ps.m, ps.u, ps.rho, V, corr,
                                     gv, soff, sidx, prm, ps.L, periodic)
    return dict(V=V, corr=corr, gv=gv, dv=dv, du=du, SF=SF, SE=SE, soff=soff, sidx=sidx)


def _clustered(seed=41, n=14):
    ps = ci.lognormal_box(n, sigma=1.5, seed=seed)
    g = np.random.default_rng(seed)
    ps.u = g.uniform(0.5, 2.0, ps.n)
    ps.v = g.normal(0, 0.3, (3, ps.n))     # strong, disordered flow: AV active
    return ps


def test_momentum_conservation(orc):
    ps = _clustered()
    r = _run(orc, ps, orc.params(64))
    tot = (ps.m * r["dv"]).sum(1)
    scale = (ps.m * r["SF"] / ps.m).sum()
    assert np.abs(tot).max() < 1e-13 * scale


def test_energy_conservation(orc):
    ps = _clustered(seed=42)
    prm = orc.params(64)
    r = _run(orc, ps, prm)
    e_th = (ps.m * r["du"]).sum()
    e_kin = (ps.m * (ps.v * r["dv"]).sum(0)).sum()
    scale = r["SE"].sum()
    assert abs(e_th + e_kin) < 1e-13 * scale
    # the viscosity does work here (the check is not trivially about P only)
    r0 = _run(orc, ps, orc.params(64, Cl=0.0, Cq=0.0))
    assert abs((ps.m * r0["du"]).sum() - e_th) > 1e-3 * abs(e_th)


def test_energy_conservation_with_expansion(orc):
    ps = _clustered(seed=43)
    prm = orc.params(64, a=0.7, adot=0.4)
    r = _run(orc, ps, prm)
    # pair sums of eqs. (mom) and (eng) cancel with weights 1/(2a^2) against
    # a^2/2: sum m du/dt + a^-4 sum xdot . m dp/dt = 0, xdot = v / a
    e_th = (ps.m * r["du"]).sum()
    e_kin = (ps.m * ((ps.v / prm["a"]) * r["dv"]).sum(0)).sum() / prm["a"] ** 4
    assert abs(e_th + e_kin) < 1e-13 * r["SE"].sum()


def test_textbook_sph_pressure_force(orc):
    """A = 1, B = 0, no viscosity: m_i dv_i/dt = -sum_j V_i V_j (P_i + P_j)
    (grad_i W(r, H_i) + grad_i W(r, H_j)) / 2."""
    ps = ci.lognormal_box(8, sigma=1.0, seed=44)
    g = np.random.default_rng(44)
    ps.u = g.uniform(0.5, 2.0, ps.n)
    n = ps.n
    corr = dict(A=np.ones(n), B=np.zeros((3, n)), gA=np.zeros((3, n)), gB=np.zeros((9, n)))
    prm = orc.params(64, Cl=0.0, Cq=0.0)
    r = _run(orc, ps, prm, corr_override=corr, gv_override=np.zeros((9, n)))
    V = r["V"]
    rho = ps.m / V
    P = (prm["gamma"] - 1) * rho * ps.u
    pos = ps.pos()
    F = np.zeros((3, n))
    h = 1e-7

    def W_of(dvec, H):
        rr = np.sqrt((dvec ** 2).sum(0))
        return orc.W(rr, H)

    for i in range(n):
        d = pos[:, i:i + 1] - pos
        d -= np.round(d)
        for Hs in (np.full(n, ps.H[i]), ps.H):
            grad = np.zeros((3, n))
            for a in range(3):
                e = np.zeros((3, 1)); e[a] = h
                grad[a] = (W_of(d + e, Hs) - W_of(d - e, Hs)) / (2 * h)
            grad[:, i] = 0.0
            F[:, i] -= 0.5 * (V[i] * V * (P[i] + P) * grad).sum(1)
    ref = F / ps.m
    assert np.abs(r["dv"] - ref).max() < 1e-6 * np.abs(ref).max()


def test_viscosity_off_for_linear_flow(orc):
    """Perfect lattice, open box, linear velocity field: grad v is exact,
    s_i = s_j so phi_VL = 1, and every pair with eta >= eta_c has a projected
    velocity difference of zero, hence Q = 0."""
    ps = ci.lattice_box(9, seed=45, jitter=0.0)
    ps.H[:] = 2.6 / 9.0                      # nearest neighbour at eta = 0.385
    G = np.array([[-0.8, 0.3, 0.1], [0.2, -0.5, 0.4], [0.0, 0.6, -0.9]])
    ps.v = G @ ps.pos()
    prm = orc.params(64, nh=3.0, eta_c=1 / 3.0, eta_f=0.2 / 3.0)
    visc = _run(orc, ps, prm, periodic=False)
    inv = _run(orc, ps, orc.params(64, nh=3.0, eta_c=1 / 3.0, eta_f=0.2 / 3.0, Cl=0.0, Cq=0.0),
               periodic=False)
    for a in range(3):
        for b in range(3):
            assert np.abs(visc["gv"][a * 3 + b] - G[a, b]).max() < 1e-12
    assert np.abs(visc["du"] - inv["du"]).max() < 1e-12 * np.abs(inv["du"]).max()
    assert np.abs(visc["dv"] - inv["dv"]).max() < 1e-12 * np.abs(inv["dv"]).max()
    # and without the projection (grad v forced to zero) the viscosity is on
    n = ps.n
    raw = _run(orc, ps, prm, periodic=False, gv_override=np.zeros((9, n)))
    assert np.abs(raw["du"] - inv["du"]).max() > 1e-3 * np.abs(inv["du"]).max()


def test_static_gas_has_no_energy_change(orc):
    ps = ci.lognormal_box(10, sigma=1.5, seed=46)
    ps.v[:] = 0.0
    r = _run(orc, ps, orc.params(64))
    assert np.all(r["du"] == 0.0)


def test_uniform_lattice_feels_no_force(orc):
    ps = ci.lattice_box(10, seed=47, jitter=0.0)
    ps.v[:] = 0.0
    r = _run(orc, ps, orc.params(64))
    assert np.abs(r["dv"]).max() < 1e-13 * (r["SF"] / ps.m).max()


def test_limiter_closed_form(orc):
    ec, ef = 0.25, 0.05
    assert orc.limiter(1.0, 1.0, 0.5, ec, ef) == 1.0          # r = 1
    assert orc.limiter(2.0, 1.0, 0.5, ec, ef) == pytest.approx(8.0 / 9.0)   # 4r/(1+r)^2 at r = 2
    assert orc.limiter(1.0, 2.0, 0.5, ec, ef) == pytest.approx(8.0 / 9.0)   # symmetric in r <-> 1/r
    assert orc.limiter(1.0, -1.0, 0.5, ec, ef) == 0.0         # r < 0
    assert orc.limiter(0.0, 1.0, 0.5, ec, ef) == 0.0          # r = 0
    assert orc.limiter(1.0, 0.0, 0.5, ec, ef) == 0.0          # r undefined
    assert orc.limiter(1.0, 1.0, 0.0, ec, ef) == pytest.approx(math.exp(-25.0))  # eta = 0
    assert orc.limiter(1.0, 1.0, ec, ec, ef) == 1.0           # continuous at eta_c
    assert orc.limiter(1.0, 1.0, ec - ef, ec, ef) == pytest.approx(math.exp(-1.0))


def test_expansion_scalings(orc):
    """With adot = 0 and no viscosity, dp/dt carries a^2 (eq. mom) and du/dt
    carries 1/(2 a^2) times xdot = v / a (eq. eng)."""
    ps = _clustered(seed=48, n=8)
    base = _run(orc, ps, orc.params(64, Cl=0.0, Cq=0.0))
    a = 0.5
    sc = _run(orc, ps, orc.params(64, Cl=0.0, Cq=0.0, a=a))
    assert np.allclose(sc["dv"], base["dv"] * a * a, rtol=1e-12, atol=0)
    assert np.allclose(sc["du"], base["du"] / a ** 3, rtol=1e-12, atol=1e-300)
