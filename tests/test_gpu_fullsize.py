"""Full-size parity on sampled outputs.

The benchmark workload (lognormal 128^3, sigma 1.5, P ~ k^-2, seed 2) in the
launch configuration the benchmark times (stored lane table, adaptive mixed
precision), and the largest single-GPU set (256^3 lognormal sigma 2.0,
P ~ k^-2.5, plus 1% of the particles in 64 dense clumps, seed 5). For a
random sample of particles the oracle evaluates every pass over the
sample's dependency rings (oracle.spot_check), and the smoothing-length
iteration for a sample (oracle.hsolve_for); the GPU outputs at the sample
must match: pair rows bit for bit, FP64 path within 1e-12, mixed path
within 1e-5, converged H within 1e-6.
"""
import numpy as np
import pytest
import torch

import crk_inputs as ci
import oracle
from paper_2202_02840_amd import CRK_FP64, CRK_MIXED_ADAPT, Context
from paper_2202_02840_amd import autotune as at
from paper_2202_02840_amd import pipeline as pl

pytestmark = pytest.mark.gpu

KEYS = ("V", "m0", "m1", "m2", "gm0", "gm1", "gm2", "A", "B", "gA", "gB", "gradv", "dpdt", "dudt")


def _at(out, perm_inv, T):
    """Sorted-order device outputs -> numpy values at original indices T."""
    k = torch.as_tensor(perm_inv[T], device="cuda")
    return {key: out[key].index_select(-1, k).double().cpu().numpy() for key in KEYS}


def _errs(got, ref):
    e = {}
    for k in KEYS:
        r = ref["dvdt" if k == "dpdt" else k]
        den = np.abs(r).max()
        e[k] = float(np.abs(got[k] - r).max() / den) if den > 0 else float(np.abs(got[k]).max())
    return e


def _errs_per_component(got, ref):
    """Worst normwise error over an output's components, each on its own scale."""
    e = {}
    for k in KEYS:
        r = ref["dvdt" if k == "dpdt" else k]
        g2, r2 = got[k].reshape(-1, r.shape[-1]), r.reshape(-1, r.shape[-1])
        worst = 0.0
        for c in range(r2.shape[0]):
            den = np.abs(r2[c]).max()
            d = np.abs(g2[c] - r2[c]).max()
            worst = max(worst, float(d / den) if den > 0 else float(d))
        e[k] = worst
    return e


def _rows_match(ctx, perm, perm_inv, T, ref_off, ref_idx):
    off, idx = ctx.export_neighbors(1)
    off = off.cpu().numpy()
    idx = idx.cpu().numpy()
    for a, t in enumerate(T):
        k = perm_inv[t]
        row = np.sort(perm[idx[off[k]:off[k + 1]]])
        if not np.array_equal(row, ref_idx[ref_off[a]:ref_off[a + 1]]):
            return int(t)
    return None


def _run(ps, prec, tuned=True, kappa=1000.0):
    ctx = Context(0)
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, prec, kappa_max=kappa)
    out = pl.step(ctx, dev, prm, count_singular=False)
    if tuned:
        cfg = at.load(prec, out["n_pairs"] / ps.n)
        if cfg:
            at.apply(ctx, cfg)
            out = pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    perm = out["perm"].long().cpu().numpy()
    perm_inv = np.empty_like(perm)
    perm_inv[perm] = np.arange(perm.shape[0])
    return ctx, out, perm, perm_inv


def test_benchmark_workload_sampled_parity():
    ps = ci.lognormal_box(128, sigma=1.5, spectral_index=-2.0, seed=2)
    g = np.random.default_rng(2024)
    T = np.sort(g.choice(ps.n, 2000, replace=False))
    print(f"[case] lognormal 128^3 n={ps.n}, sample {T.size}", flush=True)
    ref = oracle.spot_check(ps, T, oracle.params(64.0))
    print("rings", ref["rings"], flush=True)
    for prec, tol in ((CRK_FP64, 1e-12), (CRK_MIXED_ADAPT, 1e-5)):
        ctx, out, perm, perm_inv = _run(ps, prec)
        got = _at(out, perm_inv, T)
        e = _errs(got, ref)
        print(prec, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
        assert max(e.values()) <= tol, e
        # the same bar for every component of every output on its own scale
        ec = _errs_per_component(got, ref)
        print(prec, "per component", {k: f"{v:.2e}" for k, v in ec.items()}, flush=True)
        assert max(ec.values()) <= tol, ec
        if prec == CRK_FP64:
            so, si = oracle.rows_for(ps.x, ps.y, ps.z, ps.H, 1, T, ps.L)
            assert _rows_match(ctx, perm, perm_inv, T, so, si) is None
        del ctx, out
        torch.cuda.empty_cache()


def test_largest_set_sampled_parity_and_h_iteration():
    ps = ci.clustered_clump_box(256)
    g = np.random.default_rng(2025)
    # the 10^4-particle subset the full-size workload names
    T = np.sort(g.choice(ps.n, 10000, replace=False))
    print(f"[case] lognormal+clumps 256^3 n={ps.n}, sample {T.size}", flush=True)
    # every pass at the generator's supports
    ref = oracle.spot_check(ps, T, oracle.params(64.0))
    print("rings", ref["rings"], flush=True)
    ctx, out, perm, perm_inv = _run(ps, CRK_MIXED_ADAPT)
    e = _errs(_at(out, perm_inv, T), ref)
    print({k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    assert max(e.values()) <= 1e-5, e
    so, si = oracle.rows_for(ps.x, ps.y, ps.z, ps.H, 1, T, ps.L)
    assert _rows_match(ctx, perm, perm_inv, T, so, si) is None
    # the smoothing-length iteration from the generator's supports
    Hs = ctx.permute(pl.upload(ps)["H"], True)
    Hc, it, nun = ctx.hsolve(64.0, Hs, 1e-8, 1000)
    Hc = Hc.cpu().numpy()
    H_gpu = Hc[perm_inv[T]]
    H_ref, it_ref, nf = oracle.hsolve_for(ps.x, ps.y, ps.z, T, ps.H[T], 64.0, tol=1e-8,
                                          max_iter=1000, L=ps.L, H_grid=ps.H)
    print("h iterations gpu mean/max", float(it.double().mean()), int(it.max()), "unconverged", nun,
          flush=True)
    assert nun == 0 and nf == 0
    assert np.abs(H_gpu / H_ref - 1).max() < 1e-6
