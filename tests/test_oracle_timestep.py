"""Pins of the oracle's time-step terms (Sec. 3.1: the Courant criterion's
signal velocity, viscous sound speed and velocity divergence) against
closed forms and brute force that share none of its code:

* a gas at rest: no signal, no viscosity, no divergence, so v_max is the
  sound speed sqrt(gamma (gamma - 1) u) and dt_hyd = C_CFL (H / n_h) / c_s;
* two particles: approaching at closing speed s gives v_sig = s on both,
  receding gives 0, and a Hubble expansion (adot > 0, no peculiar motion) is
  never a signal;
* uniform compression v = -c (x - x0) on an open lattice: v_sig_i is c times
  the largest pair distance of i's pair set (brute force over all pairs),
  and the RK velocity gradient reproduces the linear field, so its trace is
  -3c.
"""
import math

import numpy as np

import crk_inputs as ci
import oracle


def _set(x, y, z, H, v, u=1.0):
    x, y, z, H = (np.asarray(a, dtype=np.float64) for a in (x, y, z, H))
    n = x.shape[0]
    return ci.ParticleSet(x, y, z, H, np.full(n, 1.0 / n), np.full(n, float(u)), np.asarray(v, dtype=np.float64),
                          None, L=1.0, meta=dict(kind="pin"))


def test_gas_at_rest_gives_the_sound_speed():
    ps = ci.lattice_box(8, seed=601)
    ps.v = np.zeros_like(ps.v)
    ps.u = np.full(ps.n, 2.5)
    prm = oracle.params(64.0)
    out = oracle.pipeline(ps, prm)
    assert np.all(out["vsig"] == 0.0) and np.all(out["qrho"] == 0.0)
    cs = math.sqrt(prm["gamma"] * (prm["gamma"] - 1.0) * 2.5)
    assert np.abs(out["vmax"] / cs - 1.0).max() < 1e-12
    assert np.abs(out["dt_hyd"] / (0.25 * ps.H / prm["nh"] / cs) - 1.0).max() < 1e-12


def test_two_particles_signal_velocity():
    prm = oracle.params(64.0)
    s = 0.7
    # approaching along x: closing speed s
    ps = _set([0.40, 0.50], [0.5, 0.5], [0.5, 0.5], [0.3, 0.3], [[s / 2, -s / 2], [0, 0], [0, 0]])
    out = oracle.pipeline(ps, prm, periodic=False)
    assert np.allclose(out["vsig"], s, rtol=1e-14, atol=0)
    # receding
    ps.v = -ps.v
    out = oracle.pipeline(ps, prm, periodic=False)
    assert np.all(out["vsig"] == 0.0)
    # Hubble expansion alone is no signal; peculiar motion that cancels it is not either
    ps.v = np.zeros_like(ps.v)
    out = oracle.pipeline(ps, dict(prm, a=1.0, adot=0.3), periodic=False)
    assert np.all(out["vsig"] == 0.0)
    d = ps.x[0] - ps.x[1]
    ps.v = np.array([[-0.3 * d / 2, 0.3 * d / 2], [0, 0], [0, 0]])
    out = oracle.pipeline(ps, dict(prm, a=1.0, adot=0.3), periodic=False)
    assert np.abs(out["vsig"]).max() < 1e-15


def test_uniform_compression_on_an_open_lattice():
    ps = ci.lattice_box(10, seed=602, jitter=0.2)
    c = 0.8
    ps.v = -c * (ps.pos() - 0.5)
    prm = oracle.params(64.0)
    out = oracle.pipeline(ps, prm, periodic=False)
    # brute force: N_s(i) = {j != i : r < max(H_i, H_j)} without periodic images
    P = ps.pos().T
    r = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    inset = (r < np.maximum(ps.H[:, None], ps.H[None, :])) & ~np.eye(ps.n, dtype=bool)
    rmax = np.where(inset, r, 0.0).max(axis=1)
    assert np.abs(out["vsig"] - c * rmax).max() <= 1e-12 * c
    gv = out["gradv"].reshape(9, -1)
    assert np.abs(gv[0] + gv[4] + gv[8] + 3.0 * c).max() < 1e-9


def test_time_levels_definition():
    """Levels against their definition written out differently (a log2
    formula with the boundary case checked by hand), the acceleration time
    in closed form, and the strict inequality at exact powers of two."""
    prm = oracle.params(64.0, a=1.5)
    H = np.array([0.2, 0.2, 0.2, 0.2, 0.2, 0.2])
    dv = np.zeros((3, 6))
    dv[0, 1] = 8.0            # a_hyd = 8 / 1.5^2
    dt_sub = 0.1
    # dt_hyd: plenty, exactly dt_sub/4 (must go one level deeper), tiny, huge, nan-free
    dt_hyd = np.array([1.0, 1.0, 0.025, 1e-9, 0.0999999, 0.05000001])
    dt_acc, dt_min, lev = oracle.time_levels(H, dt_hyd, dv, prm, r_soft=0.01, dt_sub=dt_sub, l_max=12)
    hh = 0.2 / prm["nh"]
    assert np.isinf(dt_acc[0])
    assert abs(dt_acc[1] - math.sqrt(min(hh, 0.01) / (8.0 / 1.5 ** 2))) < 1e-15
    assert dt_min[1] == min(1.0, dt_acc[1])
    for i in range(6):
        want = max(0, math.floor(math.log2(dt_sub / dt_min[i])) + 1) if dt_min[i] <= dt_sub else 0
        if dt_min[i] <= dt_sub and dt_sub / 2.0 ** (want - 1) < dt_min[i]:
            want -= 1
        assert lev[i] == min(want, 13), (i, lev[i], want)
    assert lev[0] == 0 and lev[2] == 3      # 0.025 == 0.1 / 4 is not > 0.1 / 4
    assert lev[3] == 13                      # beyond l_max: l_max + 1
    assert lev[4] == 1 and lev[5] == 1
