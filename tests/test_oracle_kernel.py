"""Pins of the oracle's Wendland C4 kernel (eq. C4, Sec. 2.2) against facts the
paper and calculus fix: unit normalisation, the printed prefactor, compact
support, and the derivative against finite differences."""
import math

import numpy as np
import pytest
from scipy.integrate import quad


@pytest.mark.parametrize("H", [0.3, 1.0, 2.5])
def test_kernel_integrates_to_one(orc, H):
    # SPH kernels integrate to unity (Sec. 2.2): int 4 pi r^2 W(r, H) dr = 1
    val, err = quad(lambda r: 4.0 * math.pi * r * r * float(orc.W(r, H)[()]), 0.0, H, epsabs=1e-14,
                    epsrel=1e-14, limit=200)
    assert abs(val - 1.0) < 1e-12


def test_kernel_prefactor_and_support(orc):
    # eq. C4 at eta = 0: W = 495 / (32 pi h^3)
    for H in (0.05, 1.0, 3.0):
        assert orc.W(0.0, H) * H ** 3 == pytest.approx(495.0 / (32.0 * math.pi), rel=1e-15)
        # unit extent: W = 0 for eta >= 1
        assert orc.W(H, H) == 0.0
        assert orc.W(1.5 * H, H) == 0.0
        assert orc.dWdr(H, H) == 0.0
        assert orc.dWdr(0.0, H) == 0.0


def test_kernel_monotone_positive(orc):
    r = np.linspace(0.0, 0.999, 2000)
    w = orc.W(r, np.ones_like(r))
    assert np.all(w > 0)
    assert np.all(np.diff(w) < 0)


def test_dwdr_matches_finite_differences(orc):
    H = 0.7
    r = np.linspace(0.01, 0.69, 101)
    h = 1e-6
    fd = (orc.W(r + h, np.full_like(r, H)) - orc.W(r - h, np.full_like(r, H))) / (2 * h)
    an = orc.dWdr(r, np.full_like(r, H))
    assert np.max(np.abs(fd - an)) < 1e-8 * np.max(np.abs(an))


def test_pair_gradient_matches_finite_differences(orc):
    """grad_i W(|x_i - x_j|, H_i) assembled by the oracle (RK template with
    A = 1, B = 0, gradA = gradB = 0) equals the finite-difference gradient
    of W in x_i, including the minimum image across the periodic edge."""
    rng = np.random.default_rng(5)
    n = 40
    x, y, z = rng.uniform(0, 1, (3, n))
    x[1] = x[0] + 0.97          # wrap partner of particle 0
    x[1] -= math.floor(x[1])
    H = np.full(n, 0.3)
    corr = dict(A=np.ones(n), B=np.zeros((3, n)), gA=np.zeros((3, n)), gB=np.zeros((9, n)))
    pi = np.zeros(n, dtype=np.int32)
    pj = np.arange(n, dtype=np.int32)
    WR, GR, d = orc.rk_pairs(x, y, z, H, corr, pi, pj)
    r = np.sqrt((d ** 2).sum(0))
    assert np.allclose(WR, orc.W(r, H))
    h = 1e-7
    for a in range(3):
        pos = [x.copy(), y.copy(), z.copy()]
        pos[a][0] += h
        Wp, _, _ = orc.rk_pairs(*pos, H, corr, pi, pj)
        pos[a][0] -= 2 * h
        Wm, _, _ = orc.rk_pairs(*pos, H, corr, pi, pj)
        fd = (Wp - Wm) / (2 * h)
        fd[0] = 0.0   # self pair: W(|x_i - x_i|) does not move with x_i
        assert np.max(np.abs(fd - GR[a])) < 1e-6 * max(1.0, np.max(np.abs(GR[a])))
