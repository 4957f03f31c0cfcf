"""Pins of the oracle's sampled evaluation (the per-list functions used for
full-size spot checks): the rows, the h iteration and every pass for a list
of particles must equal what the whole-set oracle computes for them."""
import numpy as np
import pytest

import crk_inputs as ci
import oracle


@pytest.fixture(scope="module")
def clumpy():
    # clustered field plus dense clumps, so supports differ by 10x and
    # more: the pair sets carry many extras (j reaching i only by H_j)
    return ci.clustered_clump_box(24, sigma=2.0, seed=31, n_clumps=4, clump_frac=0.05)


@pytest.mark.parametrize("which", [0, 1])
def test_rows_for_equal_whole_set_rows(clumpy, which):
    ps = clumpy
    off, idx = oracle.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, True, which, "grid")
    g = np.random.default_rng(5)
    T = np.sort(g.choice(ps.n, 400, replace=False))
    o2, i2 = oracle.rows_for(ps.x, ps.y, ps.z, ps.H, which, T, ps.L)
    for k, t in enumerate(T):
        assert np.array_equal(i2[o2[k]:o2[k + 1]], idx[off[t]:off[t + 1]]), t


def test_rows_for_brute_force_small():
    ps = ci.lognormal_box(12, sigma=1.5, seed=32)
    T = np.arange(ps.n)
    for which in (0, 1):
        off, idx = oracle.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, True, which, "brute")
        o2, i2 = oracle.rows_for(ps.x, ps.y, ps.z, ps.H, which, T, ps.L)
        assert np.array_equal(off, o2) and np.array_equal(idx, i2)


def test_hsolve_for_matches_whole_set_iteration(clumpy):
    ps = clumpy
    H, it, nf = oracle.hsolve(ps.x, ps.y, ps.z, ps.H, 64.0, tol=1e-12, max_iter=2000, L=ps.L)
    g = np.random.default_rng(6)
    T = np.sort(g.choice(ps.n, 300, replace=False))
    H2, it2, nf2 = oracle.hsolve_for(ps.x, ps.y, ps.z, T, ps.H[T], 64.0, tol=1e-12, max_iter=2000,
                                     L=ps.L, H_grid=ps.H)
    assert nf == 0 and nf2 == 0
    # the sums run over the same pairs in another order
    assert np.abs(H2 / H[T] - 1).max() < 1e-10


def test_spot_check_equals_whole_set_pipeline(clumpy):
    ps = clumpy
    prm = oracle.params(64.0)
    full = oracle.pipeline(ps, prm)
    g = np.random.default_rng(7)
    T = np.sort(g.choice(ps.n, 250, replace=False))
    sc = oracle.spot_check(ps, T, prm)
    assert sc["rings"][3] < ps.n or ps.n < 20000
    assert sc["n_pairs"] == int(np.diff(full["soff"])[T].sum())
    for k in ("V", "m0", "m1", "m2", "gm0", "gm1", "gm2", "A", "B", "gA", "gB", "gradv", "dvdt",
              "dudt", "SF", "SE"):
        assert np.array_equal(sc[k], full[k][..., T]), k
