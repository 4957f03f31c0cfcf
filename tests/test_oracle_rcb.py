"""Pins of the RCB leaf-tiling oracle (Sec. 3.3): closed-form leaves of a
cubic lattice, the leaf-size window N_ppl in [128, 256], the key order of
every split, and completeness of the leaf interaction lists against
brute-force neighbour pairs."""
import numpy as np
import pytest

import crk_inputs as ci
from oracle import rcb


def lattice(nside):
    g = (np.arange(nside) + 0.5) / nside
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def test_lattice_leaves_are_the_predicted_blocks():
    # 16^3 lattice: splits go x, y, z, x (largest extent, lowest axis on a
    # tie), so the 16 leaves of 256 are 4 x 8 x 8 blocks of lattice sites
    x, y, z = lattice(16)
    order, loff, boff = rcb.rcb(x, y, z, 1.0, nppl=256, bucket=32)
    assert sorted(order.tolist()) == list(range(16 ** 3))
    assert np.all(np.diff(loff) == 256)
    ix = np.floor(x * 16).astype(int)
    iy = np.floor(y * 16).astype(int)
    iz = np.floor(z * 16).astype(int)
    blocks = set()
    for k in range(16):
        mem = order[loff[k]:loff[k + 1]]
        bx, by, bz = set(ix[mem] // 4), set(iy[mem] // 8), set(iz[mem] // 8)
        assert len(bx) == len(by) == len(bz) == 1, (k, bx, by, bz)
        blocks.add((bx.pop(), by.pop(), bz.pop()))
    assert len(blocks) == 16
    # buckets of 32 inside: 4 x 4 x 2 blocks after x, y, z splits of 256
    assert np.all(np.diff(boff) == 32)


@pytest.mark.parametrize("n", [4096, 5000, 20000])
def test_leaf_sizes_in_the_paper_window(n):
    rng = np.random.default_rng(n)
    x, y, z = rng.random((3, n))
    order, loff, boff = rcb.rcb(x, y, z, 1.0, nppl=256, bucket=32)
    sizes = np.diff(loff)
    assert sizes.min() >= 128 and sizes.max() <= 256
    assert np.diff(boff).max() <= 32
    assert np.array_equal(np.sort(order), np.arange(n))
    # leaf boundaries are bucket boundaries
    assert set(loff.tolist()) <= set(boff.tolist())


def test_split_separates_keys():
    # at the root of a random set the first half (tree order) holds the
    # floor(n/2) smallest keys of the split axis, which is the largest extent
    rng = np.random.default_rng(3)
    n = 3001
    x = rng.random(n) * 0.5
    y = rng.random(n)
    z = rng.random(n) * 0.25
    order, loff, _ = rcb.rcb(x, y, z, 1.0, nppl=256, bucket=32)
    qy = rcb.keys(y, 1.0)
    left = order[: n // 2]
    right = order[n // 2:]
    assert qy[left].max() <= qy[right].min()


def test_interaction_lists_cover_every_pair():
    ps = ci.lognormal_box(16, sigma=1.5, seed=4)
    import oracle
    order, loff, _ = rcb.rcb(ps.x, ps.y, ps.z, ps.L, nppl=256, bucket=32)
    lo, hi, hm = rcb.leaf_boxes(ps.x, ps.y, ps.z, ps.H, order, loff)
    lists = rcb.interaction_lists(lo, hi, hm, ps.L)
    leaf_of = np.empty(ps.n, dtype=np.int64)
    for k in range(len(loff) - 1):
        leaf_of[order[loff[k]:loff[k + 1]]] = k
    off, idx = oracle.neighbors(ps.x, ps.y, ps.z, ps.H, L=ps.L, which=1, method="brute")
    for i in range(ps.n):
        for j in idx[off[i]:off[i + 1]]:
            assert leaf_of[j] in lists[leaf_of[i]]
    # and the lists are symmetric
    for a, row in enumerate(lists):
        for b in row:
            assert a in lists[b]


def test_batch_boxes_are_separate_trees():
    rng = np.random.default_rng(5)
    sizes = [100, 700, 300]
    off = np.concatenate([[0], np.cumsum(sizes)])
    x, y, z = rng.random((3, off[-1]))
    order, loff, _ = rcb.rcb(x, y, z, 1.0, nppl=256, bucket=32, box_offsets=off)
    for k in range(len(loff) - 1):
        mem = order[loff[k]:loff[k + 1]]
        b = np.searchsorted(off, mem, side="right") - 1
        assert len(set(b.tolist())) == 1
    # a box smaller than N_ppl is one leaf
    assert loff[1] == 100
