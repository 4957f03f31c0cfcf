"""Oracle parity at the sizes the workloads state.

* The 32^3 jittered lattice (32,768 particles, uniform H for 64
  neighbours, rho = 1 given): every output against the whole-set FP64
  oracle, FP64 path within 1e-12, both mixed modes within 1e-5.
* The 512-box batch (sides 8..48 log-uniform, half lattice, half lognormal,
  about 10.5M particles): the step recorded as one HIP graph and replayed,
  in the launch configuration the benchmark times (adaptive mixed
  precision, the stored batch lanes); boxes sampled across the size range
  against the oracle, each within 1e-5.
* CRK_MIXED (FP32 pair terms in every pass) on the clustered 128^3 workload
  against the FP64 GPU path: its documented error, far above 1e-5 there,
  next to the adaptive mode, which meets 1e-5.
"""
import numpy as np
import pytest
import torch

import crk_inputs as ci
import oracle
from gpu_helpers import OUTPUTS, compare, gpu_run, normwise, oracle_run
from paper_2202_02840_amd import CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT, Context
from paper_2202_02840_amd import autotune as at
from paper_2202_02840_amd import pipeline as pl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lattice32():
    ps = ci.lattice_box(32, seed=1)
    return ps, oracle_run(ps)


@pytest.mark.parametrize("prec,tol", [(CRK_FP64, 1e-12), (CRK_MIXED, 1e-5), (CRK_MIXED_ADAPT, 1e-5)])
def test_lattice_32_whole_set(lattice32, prec, tol):
    ps, ref = lattice32
    print(f"[case] lattice 32^3 n={ps.n} precision={prec}", flush=True)
    res = gpu_run(ps, prec)
    assert res["n_pairs"] == ref["n_pairs"]
    errs = compare(res, ref)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= tol, (k, e)


def test_512_box_batch_graph_replay_sampled_boxes():
    boxes = ci.batch_boxes(512, seed=3)
    ps, off = pl.concat(boxes)
    print(f"[case] 512 boxes n={ps.n}", flush=True)
    ctx = Context(0)
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, CRK_MIXED_ADAPT)
    io = ctx.step_buffers(dev)
    npairs, _ = ctx.step(io, prm, box_offsets=off)
    cfg = at.load(CRK_MIXED_ADAPT, npairs / ps.n, kind="batch")
    if cfg:
        at.apply(ctx, cfg)
    ctx.graph_capture(io, prm, box_offsets=off, headroom=0.25)
    for k in OUTPUTS:
        if k in io and k != "nsum":
            io[k].zero_()
    for _ in range(3):
        ctx.graph_replay(status=False)
    st, info = ctx.graph_replay()
    assert st >= 0 and info["n_pairs"] == npairs, (st, info)
    res = pl.to_original({k: io[k] for k in OUTPUTS if k in io}, io["perm"])
    sizes = np.array([b.n for b in boxes])
    order = np.argsort(sizes)
    sample = sorted(set(order[:: len(order) // 12].tolist() + [int(order[0]), int(order[-1])]))
    worst = 0.0
    for b in sample:
        ref = oracle_run(boxes[b])
        lo, hi = off[b], off[b + 1]
        for k in OUTPUTS:
            if k not in res:
                continue
            e = normwise(np.asarray(res[k])[..., lo:hi], ref[k])
            worst = max(worst, e)
            assert e <= 1e-5, (b, boxes[b].n, k, e)
    print(f"boxes checked {len(sample)}, sizes {sizes[sample].min()}..{sizes[sample].max()}, "
          f"worst {worst:.2e}", flush=True)


def test_pure_mixed_error_on_the_clustered_workload():
    ps = ci.lognormal_box(128, sigma=1.5, spectral_index=-2.0, seed=2)
    print(f"[case] lognormal 128^3 n={ps.n}: CRK_MIXED and CRK_MIXED_ADAPT vs CRK_FP64", flush=True)
    ctx = Context(0)
    dev = pl.upload(ps)
    keys = ("A", "B", "gA", "gB", "gradv", "dpdt", "dudt")
    outs = {}
    for prec in (CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT):
        o = pl.step(ctx, dev, pl.params_for(ps, 64.0, prec), count_singular=False)
        outs[prec] = {k: o[k].clone() for k in keys}
    torch.cuda.synchronize()

    def err(prec):
        return {k: ((outs[prec][k] - outs[CRK_FP64][k]).abs().max() /
                    outs[CRK_FP64][k].abs().max()).item() for k in keys}

    e_mixed, e_adapt = err(CRK_MIXED), err(CRK_MIXED_ADAPT)
    print("CRK_MIXED", {k: f"{v:.2e}" for k, v in e_mixed.items()}, flush=True)
    print("CRK_MIXED_ADAPT", {k: f"{v:.2e}" for k, v in e_adapt.items()}, flush=True)
    assert max(e_adapt.values()) <= 1e-5
    # as the header states, CRK_MIXED misses 1e-5 here: measured 3e-2 in A,
    # 3e-1 in B and grad A, grad B off by ~900x its largest value (the few
    # nearly singular m2, whose FP32 sums lose the result), 6e-1 in grad v,
    # 3e-1 in dv/dt and 2e-1 in du/dt: errors of order one in those rows,
    # which move with any change of the FP32 rounding, so only the order is
    # checked
    assert max(e_mixed.values()) > 1e-5
    assert max(e_mixed[k] for k in ("gradv", "dpdt", "dudt")) < 1.0
