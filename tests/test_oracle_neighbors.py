"""Pins of the oracle's neighbour sets: the cell-grid search against the O(N^2)
brute force (bit-exact), the brute force against an independent k-d tree,
and the structural facts of the two sets."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import crk_inputs as ci


def _sets():
    yield "lattice", ci.lattice_box(12, seed=11)
    yield "lognormal", ci.lognormal_box(16, sigma=1.5, seed=12)
    yield "tiny", ci.lognormal_box(4, sigma=1.0, seed=13, hcap=0.45)


@pytest.mark.parametrize("name,ps", list(_sets()))
@pytest.mark.parametrize("which", [0, 1])
def test_grid_equals_brute_force(orc, name, ps, which):
    b = orc.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, True, which, "brute")
    g = orc.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, True, which, "grid")
    assert np.array_equal(b[0], g[0])
    assert np.array_equal(b[1], g[1])


def test_brute_force_matches_kdtree(orc):
    ps = ci.lognormal_box(14, sigma=1.5, seed=21)
    off, idx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, 1.0, True, 0, "brute")
    pts = np.stack([ps.x, ps.y, ps.z], 1)
    tree = cKDTree(pts, boxsize=1.0)
    for i in range(0, ps.n, 7):
        row = set(idx[off[i]:off[i + 1]].tolist())
        ref = set(tree.query_ball_point(pts[i], ps.H[i]))
        # ignore pairs whose distance sits within rounding of the support edge
        sym = row ^ ref
        for j in sym:
            d = pts[i] - pts[j]
            d -= np.round(d)
            r = np.sqrt((d * d).sum())
            assert abs(r - ps.H[i]) < 1e-12 * ps.H[i], (i, j)


def test_pair_set_structure(orc):
    ps = ci.lognormal_box(12, sigma=1.5, seed=22)
    goff, gidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, 1.0, True, 0)
    soff, sidx = orc.neighbors(ps.x, ps.y, ps.z, ps.H, 1.0, True, 1)
    n = ps.n
    S = [set(sidx[soff[i]:soff[i + 1]].tolist()) for i in range(n)]
    G = [set(gidx[goff[i]:goff[i + 1]].tolist()) for i in range(n)]
    for i in range(n):
        assert i in G[i]                 # self pair in the gather set
        assert i not in S[i]
        assert G[i] - {i} <= S[i]
        for j in S[i]:
            assert i in S[j]             # symmetric pair set
            assert (j in G[i]) or (i in G[j])
        assert np.all(np.diff(sidx[soff[i]:soff[i + 1]]) > 0)
        assert np.all(np.diff(gidx[goff[i]:goff[i + 1]]) > 0)
