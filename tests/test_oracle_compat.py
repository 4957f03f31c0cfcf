"""Pins of the oracle's compatible energy update (eqs. compEng, compEng2,
Eij, ptdt, fij) against what the paper and the mathematics fix, sharing
none of its code:

* exact energy conservation: with p' = p + dt dp/dt, the thermal energy the
  pair terms hand out, sum_i m_i (Delta u_i + dt (adot/a)(3 gamma - 1) u_i),
  equals minus the change of sum_i m_i |p_i|^2 / (2 a^4) over the step, for
  any partition with f_ij + f_ji = 1; in a static and an expanding
  background (the latter pins the 1/a^4), at two step sizes;
* the entropy partition on two particles: with Delta E >= 0 the pair's energy
  is split in the ratio s_j : s_i (the cooler node heated more), with
  Delta E < 0 in the ratio s_i : s_j (the hotter node cooled more), with
  s = P / rho^gamma written out from the masses and energies;
* the same balance when the kick starts from other momenta than the
  state's (a Verlet half step: forces of one state, kick from another);
* particles without partners change only by the expansion term,
  -dt (adot/a)(3(gamma-1)+2) u, and not at all in a static background.
"""
import numpy as np
import pytest

import crk_inputs as ci
import oracle


def _two(u1, u2, m1, m2, closing):
    """Two particles mirrored about the box centre on the x axis, moving
    towards (closing > 0) or away from each other."""
    ps = ci.ParticleSet(np.array([0.45, 0.55]), np.array([0.5, 0.5]), np.array([0.5, 0.5]),
                        np.array([0.3, 0.3]), np.array([m1, m2]), np.array([u1, u2]),
                        np.array([[closing / 2, -closing / 2], [0.0, 0.0], [0.0, 0.0]]), None,
                        L=1.0, meta=dict(kind="pin"))
    return ps


@pytest.mark.parametrize("over", [{}, dict(a=1.3, adot=0.2)], ids=["static", "expanding"])
@pytest.mark.parametrize("dt", [1e-3, 2e-2])
def test_energy_is_conserved(over, dt):
    ps = ci.lognormal_box(12, sigma=1.5, seed=811)
    ps.v = ps.v * 20.0
    prm = oracle.params(64.0, gamma=ps.gamma, **over)
    a, g = prm["a"], prm["gamma"]
    out = oracle.pipeline(ps, prm, dt=dt)
    du = out["du_compat"]
    p = a * ps.v
    pp = p + dt * out["dvdt"]
    dkin = (ps.m * ((pp ** 2).sum(0) - (p ** 2).sum(0))).sum() / (2.0 * a ** 4)
    pair = ps.m * (du + dt * (prm["adot"] / a) * (3.0 * (g - 1.0) + 2.0) * ps.u)
    assert np.abs(pair).max() > 0
    assert abs(pair.sum() + dkin) <= 1e-12 * np.abs(pair).sum()


def test_energy_is_conserved_for_a_kick_from_other_momenta():
    ps = ci.lognormal_box(10, sigma=1.5, seed=813)
    ps.v = ps.v * 20.0
    prm = oracle.params(64.0, gamma=ps.gamma, a=1.2)
    a, dt = prm["a"], 5e-3
    out = oracle.pipeline(ps, prm)
    pk = a * ps.v + np.random.default_rng(814).normal(0, 0.5, ps.v.shape)
    du = oracle.compatible_energy(ps.x, ps.y, ps.z, ps.H, ps.v, ps.m, ps.u, ps.rho, out["V"], out,
                                  out["gradv"], out["soff"], out["sidx"], prm, out["dvdt"], dt,
                                  ps.L, True, pk=pk)
    pp = pk + dt * out["dvdt"]
    dkin = (ps.m * ((pp ** 2).sum(0) - (pk ** 2).sum(0))).sum() / (2.0 * a ** 4)
    pair = ps.m * du
    assert abs(pair.sum() + dkin) <= 1e-12 * np.abs(pair).sum()
    # pk = a v reproduces the plain call
    ref = oracle.compatible_energy(ps.x, ps.y, ps.z, ps.H, ps.v, ps.m, ps.u, ps.rho, out["V"], out,
                                   out["gradv"], out["soff"], out["sidx"], prm, out["dvdt"], dt,
                                   ps.L, True)
    same = oracle.compatible_energy(ps.x, ps.y, ps.z, ps.H, ps.v, ps.m, ps.u, ps.rho, out["V"], out,
                                    out["gradv"], out["soff"], out["sidx"], prm, out["dvdt"], dt,
                                    ps.L, True, pk=a * ps.v)
    assert np.array_equal(ref, same)


@pytest.mark.parametrize("closing", [0.8, -0.8], ids=["approaching", "receding"])
def test_entropy_partition_on_two_particles(closing):
    u1, u2, m1, m2 = 3.0, 0.5, 1.0, 1.7
    ps = _two(u1, u2, m1, m2, closing)
    prm = oracle.params(64.0)
    g, dt = prm["gamma"], 1e-2
    out = oracle.pipeline(ps, prm, periodic=False, dt=dt)
    du = out["du_compat"]
    # energy the pair hands to heat: minus the kinetic change (a = 1)
    pp = ps.v + dt * out["dvdt"]
    dE = -0.5 * (ps.m * ((pp ** 2).sum(0) - (ps.v ** 2).sum(0))).sum()
    assert abs(dE) > 0
    assert abs((ps.m * du).sum() - dE) <= 1e-13 * abs(dE)
    # approaching gas is compressed (heat gained), receding gas expands
    assert (dE > 0) == (closing > 0)
    # equal volumes by symmetry, so rho_1 / rho_2 = m_1 / m_2
    s1_over_s2 = (u1 / u2) * (m1 / m2) ** (1.0 - g)
    # m_1 Delta u_1 : m_2 Delta u_2 = f_12 : f_21
    share = (m1 * du[0]) / (m2 * du[1])
    want = 1.0 / s1_over_s2 if dE >= 0 else s1_over_s2
    assert abs(share / want - 1.0) <= 1e-12
    # particle 1 is the hotter one (s_1 > s_2)
    assert s1_over_s2 > 1.0
    if dE > 0:
        assert du[1] > du[0] > 0
    else:
        assert du[0] < du[1] < 0


@pytest.mark.parametrize("over", [{}, dict(a=0.7, adot=0.3)], ids=["static", "expanding"])
def test_particles_without_partners(over):
    g = np.arange(3) * (1.0 / 3.0) + 1.0 / 6.0
    X, Y, Z = (q.ravel() for q in np.meshgrid(g, g, g, indexing="ij"))
    n = X.size
    rng = np.random.default_rng(812)
    ps = ci.ParticleSet(X, Y, Z, np.full(n, 0.1), np.full(n, 1.0 / n), rng.uniform(0.5, 2.0, n),
                        rng.normal(0, 1, (3, n)), None, L=1.0, meta=dict(kind="pin"))
    prm = oracle.params(64.0, **over)
    dt = 0.05
    out = oracle.pipeline(ps, prm, dt=dt)
    assert out["n_pairs"] == 0
    want = -dt * (prm["adot"] / prm["a"]) * (3.0 * (prm["gamma"] - 1.0) + 2.0) * ps.u
    assert np.abs(out["du_compat"] - want).max() <= 1e-15 * np.abs(ps.u).max()
    if not over:
        assert np.all(out["du_compat"] == 0.0)
