"""The whole step behind one call (crk_step) and its recorded graph
(crk_graph_capture / crk_graph_replay): the same kernels as the call-by-call
sequence, so the results must agree bit for bit; replays after in-place
input updates must agree with an eager step on the same input; a batch of
boxes is checked against the oracle box by box; lists that outgrow the
recorded capacity and invalid input are reported, not run past."""
import numpy as np
import pytest
import torch

import crk_inputs as ci
import oracle
from gpu_helpers import OUTPUTS, normwise
from paper_2202_02840_amd import CRK_FP64, CRK_MIXED_ADAPT, CrkError, Context
from paper_2202_02840_amd import pipeline as pl

pytestmark = pytest.mark.gpu

KEYS = ("perm", "V", "m0", "m1", "m2", "gm0", "gm1", "gm2", "A", "B", "gA", "gB", "gradv", "dpdt",
        "dudt")


def _same(a: dict, b: dict, keys=KEYS):
    for k in keys:
        assert torch.equal(a[k], b[k]), k


def _snap(io: dict) -> dict:
    return {k: io[k].clone() for k in KEYS}


def _boxes(n_boxes=24, seed=31):
    # the C3 recipe at small sides (6..12 particles a side; below 6 a
    # lattice box's 64-neighbour support would exceed L/2)
    return ci.batch_boxes(n_boxes, seed=seed, n_min=6, n_max=12)


@pytest.mark.parametrize("prec", [CRK_FP64, CRK_MIXED_ADAPT])
def test_step_equals_call_sequence(prec):
    ps = ci.lognormal_box(16, sigma=1.5, seed=701)
    print(f"[case] crk_step vs call sequence n={ps.n} prec={prec}", flush=True)
    ctx = Context(0)
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, prec)
    ref = pl.step(ctx, dev, prm)
    io = ctx.step_buffers(dev)
    npairs, _ = ctx.step(io, prm)
    torch.cuda.synchronize()
    assert npairs == ref["n_pairs"]
    _same(io, ref)


@pytest.mark.parametrize("prec", [CRK_FP64, CRK_MIXED_ADAPT])
def test_graph_replays_match_eager(prec):
    boxes = _boxes()
    ps, off = pl.concat(boxes)
    print(f"[case] graph batch {len(boxes)} boxes n={ps.n} prec={prec}", flush=True)
    prm = pl.params_for(ps, 64.0, prec)
    dev = pl.upload(ps)
    eager = Context(0)
    ref_io = eager.step_buffers(dev)
    eager.step(ref_io, prm, box_offsets=off)

    ctx = Context(0)
    io = ctx.step_buffers(dev)
    ctx.graph_capture(io, prm, box_offsets=off, headroom=0.5)
    torch.cuda.synchronize()
    _same(io, ref_io)
    first = _snap(io)
    # every replay, with eager work and synchronisation between them
    for rep in range(3):
        for k in KEYS:
            io[k].zero_()
        st, info = ctx.graph_replay()
        assert st >= 0 and info["overflow"] == 0 and info["input_error"] == 0, info
        assert info["n_pairs"] == eager.n_pairs
        _same(io, first)
        torch.cuda.synchronize()
        print(f"replay {rep} ok", flush=True)

    # new positions and supports, written in place; the replay follows them
    g = np.random.default_rng(7)
    with torch.no_grad():
        for k in ("x", "y", "z"):
            dx = torch.as_tensor(g.uniform(-0.01, 0.01, ps.n), device="cuda")
            dev[k].copy_(torch.remainder(dev[k] + dx, 1.0))
            dev[k].masked_fill_(dev[k] >= 1.0, 0.0)
        dev["H"].mul_(1.03)
        dev["v"].mul_(1.5)
    eager.step(ref_io, prm, box_offsets=off)
    st, info = ctx.graph_replay()
    assert info["overflow"] == 0 and info["n_pairs"] == eager.n_pairs, info
    _same(io, ref_io)


def test_graph_batch_matches_oracle_per_box():
    boxes = _boxes(12, seed=33)
    ps, off = pl.concat(boxes)
    print(f"[case] graph batch vs oracle n={ps.n}", flush=True)
    prm = pl.params_for(ps, 64.0, CRK_MIXED_ADAPT)
    dev = pl.upload(ps)
    ctx = Context(0)
    io = ctx.step_buffers(dev)
    ctx.graph_capture(io, prm, box_offsets=off)
    for k in KEYS:
        io[k].zero_()
    ctx.graph_replay()
    res = pl.to_original({k: io[k] for k in KEYS if k != "perm"}, io["perm"])
    for b in (0, 3, 7, 11):
        box = boxes[b]
        lo, hi = off[b], off[b + 1]
        ref = oracle.pipeline(box, oracle.params(64.0))
        ref["dpdt"] = ref.pop("dvdt")
        for k in OUTPUTS:
            if k not in res:
                continue
            e = normwise(np.asarray(res[k])[..., lo:hi], ref[k])
            assert e <= 1e-5, (b, k, e)


def test_graph_overflow_is_reported_then_recapture():
    boxes = _boxes(8, seed=35)
    ps, off = pl.concat(boxes)
    print(f"[case] graph overflow n={ps.n}", flush=True)
    prm = pl.params_for(ps, 64.0, CRK_FP64)
    dev = pl.upload(ps)
    ctx = Context(0)
    io = ctx.step_buffers(dev)
    ctx.graph_capture(io, prm, box_offsets=off, headroom=0.0)
    with torch.no_grad():
        dev["H"].copy_(torch.clamp(dev["H"] * 1.4, max=0.45))
    st, info = ctx.graph_replay(check=False)
    assert st == -7 and info["overflow"] == 1, (st, info)
    with pytest.raises(CrkError):
        ctx.graph_replay()
    # a new recording sizes the lists for the new supports
    ctx.graph_capture(io, prm, box_offsets=off)
    eager = Context(0)
    ref_io = eager.step_buffers(dev)
    eager.step(ref_io, prm, box_offsets=off)
    st, info = ctx.graph_replay()
    assert info["overflow"] == 0
    _same(io, ref_io)


def test_graph_invalid_input_is_reported():
    boxes = _boxes(6, seed=37)
    ps, off = pl.concat(boxes)
    print(f"[case] graph invalid input n={ps.n}", flush=True)
    prm = pl.params_for(ps, 64.0, CRK_MIXED_ADAPT)
    dev = pl.upload(ps)
    ctx = Context(0)
    io = ctx.step_buffers(dev)
    ctx.graph_capture(io, prm, box_offsets=off)
    H0 = dev["H"].clone()
    x0 = dev["x"].clone()
    dev["H"][5] = float("nan")
    st, info = ctx.graph_replay(check=False)
    assert st == -2 and info["input_error"] & 1, (st, info)
    dev["H"].copy_(H0)
    dev["x"][3] = 1.5
    st, info = ctx.graph_replay(check=False)
    assert st == -1 and info["input_error"] & 2, (st, info)
    dev["x"].copy_(x0)
    dev["H"][2] = 0.6
    st, info = ctx.graph_replay(check=False)
    assert st == -3 and info["input_error"] & 8, (st, info)
    dev["H"].copy_(H0)
    st, info = ctx.graph_replay()
    assert st >= 0 and info["input_error"] == 0
    eager = Context(0)
    ref_io = eager.step_buffers(dev)
    eager.step(ref_io, prm, box_offsets=off)
    _same(io, ref_io)


def test_graph_is_dropped_when_workspace_grows():
    small = ci.lattice_box(8, seed=711)
    big = ci.lattice_box(16, seed=712)
    print("[case] graph dropped on regrowth", flush=True)
    ctx = Context(0)
    d1 = pl.upload(small)
    io = ctx.step_buffers(d1)
    ctx.graph_capture(io, pl.params_for(small, 64.0, CRK_FP64))
    ctx.graph_replay()
    d2 = pl.upload(big)
    ctx.step(ctx.step_buffers(d2), pl.params_for(big, 64.0, CRK_FP64))
    with pytest.raises(CrkError, match="STATE"):
        ctx.graph_replay()
