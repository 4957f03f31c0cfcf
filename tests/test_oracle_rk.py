"""Pins of the oracle's volume, moments and RK corrections.

The corrections are fixed by the two constraints stated with eq. (RK)
(zeroth moment 1, first moment 0). Their x_i-derivatives, with the
coefficients following x_i, give two more identities that involve every
gradient moment and every coefficient gradient:
    sum_j V_j W^R_ij = 1,           sum_j V_j x_ij W^R_ij = 0,
    sum_j V_j grad W^R_ij = 0,      sum_j V_j x_ij (x) grad W^R_ij = -I.
A dropped term, a wrong sign or a transposed index anywhere in the moments,
the solve or the eq. (gRK) template breaks at least one of them. The RK
gradient of a linear field is then exact (eq. gradv), also at free surfaces.
"""
import numpy as np
import pytest

import crk_inputs as ci


def _identities(orc, ps, periodic=True):
    goff, gidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, periodic, 0)
    _, V, _ = orc.volume(ps.x, ps.y, ps.z, ps.H, goff, gidx, ps.L, periodic)
    mom = orc.moments(ps.x, ps.y, ps.z, ps.H, V, goff, gidx, ps.L, periodic)
    corr = orc.corrections(mom)
    n = ps.n
    pi = np.repeat(np.arange(n), np.diff(goff)).astype(np.int32)
    WR, GR, d = orc.rk_pairs(ps.x, ps.y, ps.z, ps.H, corr, pi, gidx, ps.L, periodic)
    Vj = V[gidx]
    res = {}
    res["zeroth"] = np.abs(np.bincount(pi, Vj * WR, n) - 1).max()
    res["first"] = max(np.abs(np.bincount(pi, Vj * d[a] * WR, n)).max() for a in range(3)) / ps.H.max()
    scale = np.abs(np.bincount(pi, Vj * np.abs(GR[0]), n)).max()
    res["grad_zeroth"] = max(np.abs(np.bincount(pi, Vj * GR[a], n)).max() for a in range(3)) / scale
    res["grad_first"] = max(np.abs(np.bincount(pi, Vj * d[a] * GR[b], n) + (a == b)).max()
                            for a in range(3) for b in range(3))
    return res, corr, V, goff, gidx


CASES = [
    ("jittered lattice", lambda: ci.lattice_box(14, seed=31), True),
    ("lognormal clustered", lambda: ci.lognormal_box(16, sigma=1.5, seed=32), True),
    ("open box with free surface", lambda: ci.lattice_box(10, seed=33, jitter=0.2), False),
]


@pytest.mark.parametrize("name,make,periodic", CASES)
def test_reproducing_identities(orc, name, make, periodic):
    ps = make()
    if not periodic:
        ps.H = ps.H * 1.3
    res, corr, *_ = _identities(orc, ps, periodic)
    assert corr["n_singular"] == 0
    for k, v in res.items():
        # roundoff grows with the condition number of m2 on clustered sets;
        # any mistake in a term shows up at O(1)
        assert v < 1e-11, (k, v)


def test_perfect_lattice_has_no_first_moment(orc):
    ps = ci.lattice_box(10, seed=34, jitter=0.0)
    goff, gidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, 1.0, True, 0)
    nsum, V, N = orc.volume(ps.x, ps.y, ps.z, ps.H, goff, gidx)
    # all particles see the same neighbourhood: identical n_i
    assert np.ptp(nsum) < 1e-12 * nsum.mean()
    mom = orc.moments(ps.x, ps.y, ps.z, ps.H, V, goff, gidx)
    corr = orc.corrections(mom)
    assert np.abs(mom["m1"]).max() < 1e-14
    assert np.abs(corr["B"]).max() < 1e-11
    assert np.allclose(corr["A"], 1.0 / mom["m0"], rtol=1e-13)


def test_volume_continuum_limit(orc):
    # n_i approaches the number density as the support grows (Sec. 2.2)
    errs = []
    for ratio in (1.5, 2.5, 4.0):
        ps = ci.lattice_box(12, seed=35, jitter=0.0)
        ps.H[:] = ratio / 12.0
        goff, gidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, 1.0, True, 0)
        nsum, _, _ = orc.volume(ps.x, ps.y, ps.z, ps.H, goff, gidx)
        errs.append(abs(nsum[0] / ps.n - 1.0))
    assert errs[-1] < 2e-3
    assert errs[0] > errs[-1]


def test_neighbour_count_nondecreasing_in_H(orc):
    ps = ci.lognormal_box(10, sigma=1.5, seed=36)
    for i in (0, 100, 500):
        Hs = np.linspace(0.02, 0.3, 60)
        N = np.array([4 * np.pi / 3 * h ** 3 * orc.nsum_at(ps.x, ps.y, ps.z, i, h) for h in Hs])
        assert np.all(np.diff(N) >= -1e-12 * N[1:])


def test_isolated_particle_self_term(orc):
    # a lone particle's density is its own kernel value: n_i = W(0, H_i)
    x = np.array([0.1, 0.6]); y = np.array([0.1, 0.6]); z = np.array([0.1, 0.6])
    H = np.array([0.2, 0.2])
    goff, gidx = orc.neighbors(x, y, z, H, 1.0, True, 0)
    nsum, V, N = orc.volume(x, y, z, H, goff, gidx)
    assert nsum[0] == orc.W(0.0, 0.2)
    assert N[0] == pytest.approx(4 * np.pi / 3 * 495 / (32 * np.pi))   # = 20.625


def test_singular_fallback_on_a_plane(orc):
    # coplanar particles: m2 has a zero eigenvalue; normalised SPH fallback
    g = np.random.default_rng(7)
    n = 200
    x, y = g.uniform(0, 1, (2, n))
    z = np.full(n, 0.5)
    H = np.full(n, 0.25)
    goff, gidx = orc.neighbors(x, y, z, H, 1.0, True, 0)
    _, V, _ = orc.volume(x, y, z, H, goff, gidx)
    mom = orc.moments(x, y, z, H, V, goff, gidx)
    corr = orc.corrections(mom)
    assert corr["n_singular"] == n
    assert np.allclose(corr["A"], 1.0 / mom["m0"])
    assert np.all(corr["B"] == 0.0) and np.all(corr["gB"] == 0.0)


@pytest.mark.parametrize("periodic", [False])
def test_gradient_of_linear_field_is_exact(orc, periodic):
    ps = ci.lattice_box(9, seed=37, jitter=0.25)
    ps.H = ps.H * 1.3
    G = np.array([[0.3, -1.2, 0.5], [2.0, 0.1, -0.7], [-0.4, 0.9, 1.1]])
    c = np.array([0.2, -0.1, 0.05])
    v = G @ ps.pos() + c[:, None]
    res, corr, V, goff, gidx = _identities(orc, ps, periodic)
    gv = orc.gradv(ps.x, ps.y, ps.z, ps.H, v, V, corr, goff, gidx, ps.L, periodic)
    for a in range(3):
        for b in range(3):
            assert np.abs(gv[a * 3 + b] - G[a, b]).max() < 1e-12
