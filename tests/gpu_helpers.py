"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded input and compare element by element."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2202_02840_amd import CRK_FP64, CRK_MIXED, Context
from paper_2202_02840_amd import pipeline as pl

OUTPUTS = ("nsum", "V", "m0", "m1", "m2", "gm0", "gm1", "gm2", "A", "B", "gA", "gB", "gradv",
           "dpdt", "dudt")


def oracle_run(ps, nres=64.0, **over):
    prm = oracle.params(nres, gamma=ps.gamma, **over)
    out = oracle.pipeline(ps, prm)
    out["dpdt"] = out.pop("dvdt")
    return out


def gpu_run(ps, precision=CRK_FP64, nres=64.0, lanes=None, ctx=None, walk=None, **over):
    import torch
    ctx = ctx or Context(0)
    if lanes:
        ctx.set_lanes(*lanes)
    if walk:
        ctx.set_walk(*walk)
    dev = pl.upload(ps)
    p = pl.params_for(ps, nres, precision, **over)
    out = pl.step(ctx, dev, p)
    torch.cuda.synchronize()
    res = pl.to_original(out, out["perm"])
    res["ctx"] = ctx
    return res


def normwise(y, ref):
    """max |y - ref| / max |ref| over every element of one output."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    num = np.abs(y - ref).max()
    if den == 0.0:
        return float(num)
    return float(num / den)


def compare(res, ref, keys=OUTPUTS, skip_rows=None):
    errs = {}
    for k in keys:
        y, r = np.asarray(res[k]), np.asarray(ref[k])
        if skip_rows is not None and skip_rows.any():
            keep = ~skip_rows
            y, r = y[..., keep], r[..., keep]
        errs[k] = normwise(y, r)
    return errs


def rows_original(off, idx, perm):
    """GPU CSR (sorted indices) -> per-row sorted original indices."""
    off = off.cpu().numpy()
    idx = idx.cpu().numpy()
    p = perm.cpu().numpy().astype(np.int64)
    n = p.shape[0]
    rows = [None] * n
    for k in range(n):
        rows[p[k]] = np.sort(p[idx[off[k]:off[k + 1]]])
    return rows
