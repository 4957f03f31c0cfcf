"""Pins of the oracle's viscous pressure (eqs. visc, mu), of the pressure that
eq. (eng) attributes to each side of a pair, and of the network's input
features, on cases whose values follow from the printed equations alone.

Two particles in an open box, with the RK coefficients forced to A = 1,
B = 0 (so grad W^R is the plain kernel gradient) and grad v forced to zero
(so s_i = s_j = 0, the limiter is 0 and the projected velocity difference of
eq. hatvi is the raw one, v_i - v_j + adot d). For the pair (1, 2),
D_1 = grad W^R_21 - grad W^R_12 = -D_2, and

  m_1 dp_1/dt = (a^2/2) V_1 V_2 (P_1 + Q_1 + P_2 + Q_2) D_1           (eq. mom)
  m_1 du_1/dt = (1/(2a^2)) V_1 V_2 (P_2 + Q_2) (xdot_2 - xdot_1).D_1  (eq. eng)
  m_2 du_2/dt = (1/(2a^2)) V_1 V_2 (P_1 + Q_1) (xdot_1 - xdot_2).D_2

so the ratios of the viscous to the inviscid outputs give Q_1 + Q_2 (from
either particle's dp/dt) and Q_2 and Q_1 separately (from du_1/dt and
du_2/dt), whatever the kernel, the volumes or D are. Those are compared with
Q_k = rho_k (-C_l c_k mu_k + C_q mu_k^2), mu_k = min(0, (hh_k/a) (uhat.d) /
(r^2 + hh_k^2 eps^2)), hh_k = H_k / n_h, c_k = sqrt(gamma P_k / rho_k),
evaluated here from the numbers of the case. The inputs are chosen so that
hh != H, eps^2 != eps, c_k != |mu_k| (C_l and C_q not interchangeable),
P_1 != P_2, rho_1 != rho_2 and a != 1.
"""
import math

import numpy as np
import pytest

import crk_inputs as ci


def _two(v1=(0.4, 0.1, -0.05), v2=(-0.3, 0.05, 0.02)):
    r = 0.08
    x = np.array([0.5 - r / 2, 0.5 + r / 2])
    y = np.array([0.5, 0.5])
    z = np.array([0.5, 0.5])
    ps = ci.ParticleSet(x=x, y=y, z=z, H=np.array([0.3, 0.22]), m=np.array([0.01, 0.025]),
                        u=np.array([0.6, 2.3]), v=np.array([v1, v2]).T.copy(),
                        rho=np.array([1.3, 0.6]), L=1.0)
    return ps


def _eval(orc, ps, prm):
    n = ps.n
    goff, gidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, False, 0)
    soff, sidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, False, 1)
    _, V, _ = orc.volume(ps.x, ps.y, ps.z, ps.H, goff, gidx, ps.L, False)
    corr = dict(A=np.ones(n), B=np.zeros((3, n)), gA=np.zeros((3, n)), gB=np.zeros((9, n)))
    ts = {}
    dv, du, _, _ = orc.derivatives(ps.x, ps.y, ps.z, ps.H, ps.v, ps.m, ps.u, ps.rho, V, corr,
                                   np.zeros((9, n)), soff, sidx, prm, ps.L, False, ts=ts)
    assert int(soff[-1]) == 2      # each particle has the other as its only partner
    return dv, du, ts


def _expected_Q(ps, prm):
    """Q_1, Q_2 of eqs. (visc), (mu) for the two-particle case, written out."""
    g = prm["gamma"]
    d = np.array([ps.x[0] - ps.x[1], ps.y[0] - ps.y[1], ps.z[0] - ps.z[1]])
    r2 = float(d @ d)
    uhat = ps.v[:, 0] - ps.v[:, 1] + prm["adot"] * d      # limiter 0: no projection
    ud = float(uhat @ d)
    Q = []
    for k in (0, 1):
        P = (g - 1.0) * ps.rho[k] * ps.u[k]
        c = math.sqrt(g * P / ps.rho[k])
        hh = ps.H[k] / prm["nh"]
        mu = min(0.0, (hh / prm["a"]) * ud / (r2 + hh * hh * prm["eps"] ** 2))
        Q.append(ps.rho[k] * (-prm["Cl"] * c * mu + prm["Cq"] * mu * mu))
    P = [(g - 1.0) * ps.rho[k] * ps.u[k] for k in (0, 1)]
    return Q, P, ud


@pytest.mark.parametrize("a,adot", [(1.0, 0.0), (0.8, 0.3)])
def test_viscous_pressure_two_particles(orc, a, adot):
    ps = _two()
    prm = orc.params(64, a=a, adot=adot)
    inv = orc.params(64, a=a, adot=adot, Cl=0.0, Cq=0.0)
    Q, P, ud = _expected_Q(ps, prm)
    assert ud < 0.0 and Q[0] > 0.0 and Q[1] > 0.0          # approaching: viscosity on
    assert abs(Q[0] - Q[1]) > 0.1 * Q[0]                   # distinct sides
    dv, du, ts = _eval(orc, ps, prm)
    dv0, du0, _ = _eval(orc, ps, inv)
    # eq. (mom): every component of both particles carries (P1+Q1+P2+Q2)/(P1+P2)
    ratio_m = (P[0] + Q[0] + P[1] + Q[1]) / (P[0] + P[1])
    for k in (0, 1):
        assert dv0[0, k] != 0.0
        assert dv[0, k] / dv0[0, k] == pytest.approx(ratio_m, rel=1e-12)
    # eq. (eng): particle 1's energy carries particle 2's P + Q, and vice versa
    assert du[0] / du0[0] == pytest.approx((P[1] + Q[1]) / P[1], rel=1e-12)
    assert du[1] / du0[1] == pytest.approx((P[0] + Q[0]) / P[0], rel=1e-12)
    # time-step term: the largest Q_i / rho_i over i's pairs
    assert ts["qrho"][0] == pytest.approx(Q[0] / ps.rho[0], rel=1e-12)
    assert ts["qrho"][1] == pytest.approx(Q[1] / ps.rho[1], rel=1e-12)


def test_energy_attribution_without_viscosity(orc):
    """eq. (eng) weights i's energy change by P_j: with no viscosity,
    m_1 du_1/dt : m_2 du_2/dt = P_2 : P_1 (the kinetic factors are equal)."""
    ps = _two()
    prm = orc.params(64, Cl=0.0, Cq=0.0)
    _, du, _ = _eval(orc, ps, prm)
    P = (prm["gamma"] - 1.0) * ps.rho * ps.u
    assert P[0] / P[1] < 0.8                                 # unequal pressures
    assert (ps.m[0] * du[0]) / (ps.m[1] * du[1]) == pytest.approx(P[1] / P[0], rel=1e-12)


def test_receding_pair_has_no_viscosity(orc):
    """mu = min(0, ...): a receding pair gets Q = 0 on both sides."""
    ps = _two(v1=(-0.4, 0.1, -0.05), v2=(0.3, 0.05, 0.02))
    prm = orc.params(64)
    dv, du, ts = _eval(orc, ps, prm)
    dv0, du0, _ = _eval(orc, ps, orc.params(64, Cl=0.0, Cq=0.0))
    assert np.array_equal(dv, dv0) and np.array_equal(du, du0)
    assert np.all(ts["qrho"] == 0.0)


def test_viscosity_constants_enter_as_printed(orc):
    """C_l scales the term linear in mu and C_q the quadratic one: Q from
    (C_l, C_q) = (2, 0) plus Q from (0, 1) is Q from (2, 1)."""
    ps = _two()
    out = {}
    for cl, cq in ((2.0, 1.0), (2.0, 0.0), (0.0, 1.0), (0.0, 0.0)):
        out[(cl, cq)] = _eval(orc, ps, orc.params(64, Cl=cl, Cq=cq))[1]
    base = out[(0.0, 0.0)]
    lin = out[(2.0, 0.0)] - base
    quad = out[(0.0, 1.0)] - base
    both = out[(2.0, 1.0)] - base
    assert np.allclose(lin + quad, both, rtol=1e-12, atol=0)
    Q_lin, P, _ = _expected_Q(ps, orc.params(64, Cl=2.0, Cq=0.0))
    Q_quad, _, _ = _expected_Q(ps, orc.params(64, Cl=0.0, Cq=1.0))
    # particle 1's energy: (P2 + Q2) / P2 - 1 = Q2 / P2
    assert lin[0] / base[0] == pytest.approx(Q_lin[1] / P[1], rel=1e-12)
    assert quad[0] / base[0] == pytest.approx(Q_quad[1] / P[1], rel=1e-12)
    # the linear and quadratic parts differ here, so swapping C_l and C_q shows
    assert abs(Q_lin[1] / 2.0 - Q_quad[1]) > 0.1 * Q_quad[1]


# ---------------------------------------------------------------- features
@pytest.mark.parametrize("nside", [12, 17])      # 17^3 > 4096 takes the oracle's grid path
def test_features_brute_force(orc, nside):
    ps = ci.lognormal_box(nside, sigma=1.5, seed=61)
    # a spread of starting supports, as the iteration sees them
    g = np.random.default_rng(61)
    H = ps.H * np.exp(g.uniform(-0.4, 0.4, ps.n))
    ps.H = np.minimum(H, 0.45)
    f = orc.hnet_features(ps.x, ps.y, ps.z, ps.H, 64.0, ps.L)
    sample = np.arange(0, ps.n, max(1, ps.n // 300))
    ref = _brute_features_rows(orc, ps, 64.0, sample)
    assert np.allclose(f[:, sample], ref, rtol=1e-12, atol=1e-12)


def _brute_features_rows(orc, ps, Nres, rows):
    """The eight network inputs of the listed particles from brute-force
    distances (minimum image): N_w(h) = (4 pi/3) h^3 sum_{r<h} W(r, h) (eq.
    hi), n_raw(h) = #{r < h}, self included in both."""
    pos = ps.pos()
    n = ps.n
    out = np.empty((8, len(rows)))
    for c, i in enumerate(rows):
        d = pos[:, i:i + 1] - pos
        d -= ps.L * np.round(d / ps.L)
        r = np.sqrt((d * d).sum(0))
        h = ps.H[i]

        def Nw(hh):
            sel = r < hh
            return 4.0 / 3.0 * math.pi * hh ** 3 * orc.W(r[sel], hh).sum()

        out[0, c] = math.log(Nw(h) / Nres)
        out[1, c] = (Nres / Nw(h)) ** (1.0 / 3.0) - 1.0
        out[2, c] = math.log(8.0 * Nw(h / 2) / Nres)
        out[3, c] = math.log(64.0 * Nw(h / 4) / Nres)
        out[4, c] = math.log(float((r < h).sum()) / Nres)
        out[5, c] = math.log(8.0 * float((r < h / 2).sum()) / Nres)
        out[6, c] = math.log(h * n ** (1.0 / 3.0) / ps.L)
        out[7, c] = 1.0
    return out


def test_features_match_eq_hi_count(orc):
    """f0 is ln(N_i / N_res) with N_i = (4 pi/3) H^3 n_i of eq. (hi), the same
    count the smoothing-length iteration drives to N_res; f2 and f3 are that
    count at H/2 and H/4 scaled to the volume of radius H."""
    ps = ci.lognormal_box(10, sigma=1.0, seed=62)
    f = orc.hnet_features(ps.x, ps.y, ps.z, ps.H, 64.0, ps.L)
    for i in (0, 17, 333, 999):
        for col, scale in ((0, 1.0), (2, 0.5), (3, 0.25)):
            h = ps.H[i] * scale
            nsum = orc.nsum_at(ps.x, ps.y, ps.z, i, h, ps.L)
            N = 4.0 / 3.0 * math.pi * h ** 3 * nsum
            assert f[col, i] == pytest.approx(math.log(N / scale ** 3 / 64.0), rel=1e-12, abs=1e-12)
