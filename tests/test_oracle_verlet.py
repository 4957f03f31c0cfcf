"""Pins of the oracle's velocity-Verlet hydro step (eq. verletOP) against
closed forms and the integrator's known order, sharing none of its code:

* particles without partners feel no force: p and u stay, and x moves by
  p dt / a^2 = v dt / a, wrapped into the periodic box;
* a gas at rest on a perfect lattice with uniform energy stays at rest;
* second-order convergence: an inviscid (C_l = C_q = 0) clustered gas
  integrated to a fixed time with dt, dt/2 and dt/4 against a dt/16 run
  shows errors falling by ~4 per halving, in a static and an expanding
  (a = 1.3) background; dropping a half kick, kicking with the start
  derivatives only, or a wrong drift factor makes the scheme first order
  or inconsistent and fails these.
"""
import numpy as np
import pytest

import crk_inputs as ci
import oracle


def _isolated(seed):
    g = np.arange(3) * (1.0 / 3.0) + 1.0 / 6.0
    X, Y, Z = (q.ravel() for q in np.meshgrid(g, g, g, indexing="ij"))
    n = X.size
    rng = np.random.default_rng(seed)
    return ci.ParticleSet(X, Y, Z, np.full(n, 0.05), np.full(n, 1.0 / n), rng.uniform(0.5, 2.0, n),
                          rng.normal(0, 1.0, (3, n)), None, L=1.0, meta=dict(kind="pin"))


@pytest.mark.parametrize("over", [{}, dict(a=1.3)], ids=["static", "a=1.3"])
def test_free_streaming_without_partners(over):
    ps = _isolated(901)
    prm = oracle.params(64.0, **over)
    dt = 0.03
    end, d1 = oracle.verlet_step(ps, prm, dt)
    assert d1["n_pairs"] == 0
    # p = a v is unchanged (v only through the rounding of (a v) / a)
    assert np.abs(end.v - ps.v).max() <= 1e-15 * np.abs(ps.v).max()
    assert np.array_equal(end.u, ps.u)
    a = prm["a"]
    for got, x0, vc in ((end.x, ps.x, ps.v[0]), (end.y, ps.y, ps.v[1]), (end.z, ps.z, ps.v[2])):
        want = np.mod(x0 + vc * dt / a, 1.0)
        assert np.abs(got - want).max() < 1e-15
        assert np.all((got >= 0.0) & (got < 1.0))


def test_gas_at_rest_on_a_lattice_stays():
    ps = ci.lattice_box(8, seed=902, jitter=0.0)
    ps.v = np.zeros_like(ps.v)
    ps.u = np.full(ps.n, 1.5)
    prm = oracle.params(64.0, gamma=ps.gamma)
    end, d1 = oracle.verlet_step(ps, prm, 0.01)
    assert np.abs(d1["dvdt"]).max() < 1e-10
    assert np.abs(end.x - ps.x).max() < 1e-13 and np.abs(end.u - ps.u).max() < 1e-12


def _run(ps, prm, T, nsteps):
    dt = T / nsteps
    st, d = ps, None
    for _ in range(nsteps):
        st, d = oracle.verlet_step(st, prm, dt, d0=d)
    return st


def _err(a, b, L=1.0):
    dx = [np.abs((p - q + 0.5 * L) % L - 0.5 * L).max() for p, q in ((a.x, b.x), (a.y, b.y), (a.z, b.z))]
    return max(max(dx), np.abs(a.u - b.u).max(), np.abs(a.v - b.v).max())


@pytest.mark.parametrize("over", [{}, dict(a=1.3)], ids=["static", "a=1.3"])
def test_second_order_convergence(over):
    ps = ci.lognormal_box(6, sigma=0.8, seed=903)
    ps.v = ps.v * 2.0
    prm = oracle.params(64.0, gamma=ps.gamma, Cl=0.0, Cq=0.0, **over)
    T = 0.02
    ref = _run(ps, prm, T, 64)
    errs = [_err(_run(ps, prm, T, k), ref) for k in (4, 8, 16)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    print(errs, r1, r2)
    assert errs[0] > 1e-9
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5


def _energy(st, a):
    return (st.m * (st.u + ((a * st.v) ** 2).sum(0) / (2.0 * a ** 4))).sum()


@pytest.mark.parametrize("over", [{}, dict(a=1.3)], ids=["static", "a=1.3"])
def test_compatible_mode_conserves_energy_exactly(over):
    """With each half kick's energy from the compatible update, the total
    energy sum m (u + |p|^2 / (2 a^4)) is conserved to rounding over many
    steps, shocks and viscosity included (adot = 0); the du/dt mode drifts."""
    ps = ci.lognormal_box(8, sigma=1.5, seed=904)
    ps.v = ps.v * 20.0
    prm = oracle.params(64.0, gamma=ps.gamma, **over)
    a, dt = prm["a"], 2e-3
    e0 = _energy(ps, a)
    drift = {}
    for mode in ("compat", "eng"):
        st, d = ps, None
        for _ in range(6):
            st, d = oracle.verlet_step(st, prm, dt, d0=d, energy=mode)
        drift[mode] = abs(_energy(st, a) - e0) / e0
    print(drift)
    assert drift["compat"] < 1e-13
    assert drift["eng"] > 1e3 * drift["compat"]


def test_compatible_mode_is_second_order():
    ps = ci.lognormal_box(6, sigma=0.8, seed=905)
    ps.v = ps.v * 2.0
    prm = oracle.params(64.0, gamma=ps.gamma, Cl=0.0, Cq=0.0)
    T = 0.02

    def run(nsteps):
        st, d = ps, None
        for _ in range(nsteps):
            st, d = oracle.verlet_step(st, prm, T / nsteps, d0=d, energy="compat")
        return st

    ref = run(64)
    errs = [_err(run(k), ref) for k in (4, 8, 16)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    print(errs, r1, r2)
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5
