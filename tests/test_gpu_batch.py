"""Batched boxes (one build, one launch per pass over all boxes) against the
oracle run box by box: neighbour sets bit-exact per box (no pair crosses a
box), FP64 outputs within 1e-12, adaptive mixed within 1e-5."""
import numpy as np
import pytest
import torch

import crk_inputs as ci
import oracle
from gpu_helpers import OUTPUTS, normwise, rows_original
from paper_2202_02840_amd import CRK_FP64, CRK_MIXED_ADAPT, Context
from paper_2202_02840_amd import pipeline as pl

pytestmark = pytest.mark.gpu


def _boxes():
    bs = [ci.lattice_box(8, seed=601), ci.lognormal_box(10, sigma=1.5, seed=602),
          ci.lattice_box(12, seed=603, rho0=3.0, u0=0.2), ci.lognormal_box(9, sigma=1.0, seed=604),
          ci.lognormal_box(5, sigma=1.0, seed=605, hcap=0.45)]
    for k, b in enumerate(bs):
        b.u = np.full(b.n, 0.5 + k)
        b.rho = None
    return bs


@pytest.mark.parametrize("prec,tol", [(CRK_FP64, 1e-12), (CRK_MIXED_ADAPT, 1e-5)])
def test_batch_matches_per_box_oracle(prec, tol):
    boxes = _boxes()
    ps, off = pl.concat(boxes)
    print(f"[case] batch of {len(boxes)} boxes, n={ps.n}, prec={prec}", flush=True)
    ctx = Context(0)
    dev = pl.upload(ps)
    out = pl.step(ctx, dev, pl.params_for(ps, 64.0, prec), box_offsets=off)
    torch.cuda.synchronize()
    res = pl.to_original(out, out["perm"])
    o1, i1 = ctx.export_neighbors(1)
    rows = rows_original(o1, i1, ctx.perm)
    total = 0
    for b, box in enumerate(boxes):
        lo, hi = off[b], off[b + 1]
        ref = oracle.pipeline(box, oracle.params(64.0))
        ref["dpdt"] = ref.pop("dvdt")
        total += ref["n_pairs"]
        for i in range(box.n):
            assert np.array_equal(rows[lo + i] - lo, ref["sidx"][ref["soff"][i]:ref["soff"][i + 1]])
        for k in OUTPUTS:
            e = normwise(np.asarray(res[k])[..., lo:hi], ref[k])
            assert e <= tol, (b, k, e)
    assert out["n_pairs"] == total
