"""GPU parity of the Courant time-step terms (Sec. 3.1) fused into the
derivative pass: per particle the largest closing speed over the pair set,
the viscous sound speed from the largest Q_i / rho_i, v_max and dt_hyd, each
against the oracle (FP64 path 1e-12, mixed paths 1e-5, normwise), in a
static and an expanding background; a recorded step keeps the terms; the
call without the terms is refused."""
import numpy as np
import pytest
import torch

import crk_inputs as ci
import oracle
from gpu_helpers import normwise
from paper_2202_02840_amd import CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT, Context, CrkError
from paper_2202_02840_amd import pipeline as pl

pytestmark = pytest.mark.gpu

KEYS = ("vsig", "csq", "vmax", "dt_hyd")


def _ref(ps, **over):
    prm = oracle.params(64.0, gamma=ps.gamma, **over)
    out = oracle.pipeline(ps, prm)
    out["csq"] = np.sqrt(4.0 * out["qrho"])
    return out


def _gpu(ps, prec, ctx=None, **over):
    ctx = ctx or Context(0)
    dev = pl.upload(ps)
    out = pl.step(ctx, dev, pl.params_for(ps, 64.0, prec, **over), timestep=True)
    torch.cuda.synchronize()
    return pl.to_original({k: out[k] for k in KEYS}, out["perm"])


@pytest.mark.parametrize("over", [{}, dict(a=1.3, adot=0.2)], ids=["static", "expanding"])
def test_timestep_terms_match_oracle(over):
    ps = ci.lognormal_box(16, sigma=1.5, seed=801)
    ps.v = ps.v * 20.0   # strong enough flow for shocks: viscosity and signals active
    print(f"[case] timestep n={ps.n} {over}", flush=True)
    ref = _ref(ps, **over)
    assert ref["vsig"].max() > 0 and ref["qrho"].max() > 0
    for prec, tol in ((CRK_FP64, 1e-12), (CRK_MIXED_ADAPT, 1e-5), (CRK_MIXED, 1e-5)):
        got = _gpu(ps, prec, **over)
        errs = {k: normwise(got[k], ref[k]) for k in KEYS}
        print(prec, {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
        assert max(errs.values()) <= tol, (prec, errs)


def test_recorded_step_keeps_the_terms():
    boxes = ci.batch_boxes(6, seed=803, n_min=6, n_max=10)
    ps, off = pl.concat(boxes)
    print(f"[case] timestep graph n={ps.n}", flush=True)
    prm = pl.params_for(ps, 64.0, CRK_MIXED_ADAPT)
    dev = pl.upload(ps)
    eager = Context(0)
    eager.set_timestep(True)
    ref_io = eager.step_buffers(dev)
    eager.step(ref_io, prm, box_offsets=off)
    ctx = Context(0)
    ctx.set_timestep(True)
    io = ctx.step_buffers(dev)
    ctx.graph_capture(io, prm, box_offsets=off)
    ctx.graph_replay()

    def terms(c, b):
        perm = b["perm"].long()
        s = lambda k: dev[k].index_select(0, perm) if dev.get(k) is not None else None
        return c.timestep(prm, s("u"), s("m"), s("rho"), b["V"], b["gradv"])

    a, r = terms(ctx, io), terms(eager, ref_io)
    for k in KEYS:
        assert torch.equal(a[k], r[k]), k


def test_terms_need_a_derivative_call_with_them_on():
    ps = ci.lattice_box(8, seed=804)
    ctx = Context(0)
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, CRK_FP64)
    out = pl.step(ctx, dev, prm)
    with pytest.raises(CrkError) as e:
        ctx.timestep(prm, dev["u"], dev["m"], dev["rho"], out["V"], out["gradv"])
    assert e.value.status == -6


def test_time_levels_match_oracle():
    ps = ci.lognormal_box(16, sigma=1.5, seed=805)
    ps.v = ps.v * 20.0
    print(f"[case] time levels n={ps.n}", flush=True)
    ref = _ref(ps)
    prm_o = oracle.params(64.0, gamma=ps.gamma)
    dt_sub = 8.0 * float(np.median(ref["dt_hyd"]))
    r_soft = 0.5 * float(np.median(ps.H)) / prm_o["nh"]
    l_max = 5
    # the accelerations scaled up 30x (same scaling on both sides) so
    # that the acceleration criterion binds for part of the particles
    sc = 30.0
    r_acc, r_min, r_lev = oracle.time_levels(ps.H, ref["dt_hyd"], sc * ref["dvdt"], prm_o, r_soft,
                                             dt_sub, l_max)
    assert 0 < (r_lev > l_max).sum() < ps.n and len(set(r_lev.tolist())) > 3
    assert 0 < (r_min < ref["dt_hyd"]).sum() < ps.n
    # levels whose dt_min sits within 1e-5 of a boundary may differ in the mixed paths
    edges = dt_sub / 2.0 ** np.arange(l_max + 1)
    near = (np.abs(r_min[:, None] / edges[None, :] - 1.0) < 1e-5).any(1)
    for prec, tol in ((CRK_FP64, 1e-12), (CRK_MIXED_ADAPT, 1e-5)):
        ctx = Context(0)
        dev = pl.upload(ps)
        prm = pl.params_for(ps, 64.0, prec)
        out = pl.step(ctx, dev, prm, timestep=True)
        lv = ctx.time_levels(prm, out["dt_hyd"], sc * out["dpdt"], r_soft, dt_sub, l_max)
        torch.cuda.synchronize()
        got = pl.to_original({k: lv[k] for k in ("dt_acc", "dt_min", "level")}, out["perm"])
        fin = np.isfinite(r_acc)
        assert np.array_equal(np.isfinite(got["dt_acc"]), fin)
        assert normwise(got["dt_acc"][fin], r_acc[fin]) <= tol
        assert normwise(got["dt_min"], r_min) <= tol
        if prec == CRK_FP64:
            assert np.array_equal(got["level"], r_lev)
            assert lv["n_over"] == int((r_lev > l_max).sum())
        else:
            assert np.array_equal(got["level"][~near], r_lev[~near])
        print(prec, "levels", np.bincount(got["level"]).tolist(), flush=True)
