"""Recursive coordinate bisection (RCB) of a particle set into flat leaves:
the oracle of the library's leaf tiling (test infrastructure only).

Sec. 3.3 (short-range solvers) organises the particles of a domain by a
recursive coordinate bisection tree whose leaves hold N_ppl particles, and
builds interaction lists between leaves whose bounding boxes, grown by the
smoothing support, overlap. The paper does not fix the tie rules, so this
module states them (a reading recorded with the design notes):

* a coordinate is compared as the 32-bit fixed-point key
  q = floor(x / L * 2^32) (clamped to 2^32 - 1), ties broken by the
  particle's original index;
* a node with more than `bucket` particles is split along the axis of
  largest key extent (q_max - q_min; the lowest axis wins a tie), the first
  floor(n / 2) particles in key order going left;
* a leaf is the first node on a root-to-bucket path with at most `nppl`
  particles; buckets (at most `bucket` particles) refine the order inside a
  leaf, and inside a bucket particles follow the x key.

Plain recursion over index arrays, NumPy only; nothing here is shared with
the GPU library.
"""
from __future__ import annotations

import numpy as np


def keys(x, L):
    """32-bit fixed-point key of coordinates in [0, L)."""
    q = np.floor(np.asarray(x, dtype=np.float64) / L * 4294967296.0)
    return np.minimum(q, 4294967295.0).astype(np.uint64)


def rcb(x, y, z, L=1.0, nppl=256, bucket=32, box_offsets=None):
    """Leaf tiling of the particles (each box of a batch is its own tree).

    Returns (order, leaf_off, bucket_off): order[k] = original index of the
    k-th particle in tree order; leaf k holds order[leaf_off[k]:leaf_off[k+1]],
    bucket k order[bucket_off[k]:bucket_off[k+1]].
    """
    n = len(x)
    q = np.stack([keys(x, L), keys(y, L), keys(z, L)])
    if box_offsets is None:
        box_offsets = [0, n]
    order, leaves, buckets = [], [0], [0]

    def split(idx, in_leaf):
        m = len(idx)
        leaf_here = not in_leaf and m <= nppl
        if m <= bucket:
            # a bucket: particles in x-key order (ties by index)
            o = idx[np.lexsort((idx, q[0, idx]))]
            order.extend(o.tolist())
            buckets.append(buckets[-1] + m)
            if leaf_here:
                leaves.append(leaves[-1] + m)
            return
        ext = [int(q[a, idx].max()) - int(q[a, idx].min()) for a in range(3)]
        a = int(np.argmax(ext))   # first maximum: lowest axis on a tie
        o = idx[np.lexsort((idx, q[a, idx]))]
        h = m // 2
        split(o[:h], in_leaf or leaf_here)
        split(o[h:], in_leaf or leaf_here)
        if leaf_here:
            leaves.append(leaves[-1] + m)

    for b in range(len(box_offsets) - 1):
        idx = np.arange(box_offsets[b], box_offsets[b + 1], dtype=np.int64)
        if len(idx):
            split(idx, False)
    return np.asarray(order, dtype=np.int64), np.asarray(leaves, dtype=np.int64), \
        np.asarray(buckets, dtype=np.int64)


def leaf_boxes(x, y, z, H, order, leaf_off):
    """FP64 bounding box (lo[3], hi[3]) and largest support of every leaf."""
    P = np.stack([x, y, z])[:, order]
    Ho = np.asarray(H)[order]
    nl = len(leaf_off) - 1
    lo, hi, hmax = np.empty((nl, 3)), np.empty((nl, 3)), np.empty(nl)
    for k in range(nl):
        s = slice(leaf_off[k], leaf_off[k + 1])
        lo[k] = P[:, s].min(axis=1)
        hi[k] = P[:, s].max(axis=1)
        hmax[k] = Ho[s].max()
    return lo, hi, hmax


def box_gap(lo_a, hi_a, lo_b, hi_b, L):
    """Smallest distance between two axis-aligned boxes in a periodic cube
    (per axis the nearest of the three images of b)."""
    g2 = 0.0
    for a in range(3):
        best = np.inf
        for s in (-L, 0.0, L):
            g = max(0.0, lo_b[a] + s - hi_a[a], lo_a[a] - (hi_b[a] + s))
            best = min(best, g)
        g2 += best * best
    return np.sqrt(g2)


def interaction_lists(lo, hi, hmax, L, leaf_box=None):
    """Per leaf, the leaves (itself included) whose boxes come within
    max(Hmax_a, Hmax_b) + 1e-9 L of its box (the margin, far above any
    rounding of the gap, keeps the lists complete): every pair of N_s lies
    in such a leaf pair. leaf_box: box id of each leaf (leaves of different
    boxes never interact)."""
    nl = len(hmax)
    out = []
    for a in range(nl):
        row = []
        for b in range(nl):
            if leaf_box is not None and leaf_box[a] != leaf_box[b]:
                continue
            if box_gap(lo[a], hi[a], lo[b], hi[b], L) < max(hmax[a], hmax[b]) + 1e-9 * L:
                row.append(b)
        out.append(row)
    return out
