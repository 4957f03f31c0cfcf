"""GPU parity of the smoothing-length iteration (eqs. hi, thacker) against the
oracle: both iterate each particle to |dH| <= 1e-7 H from the same start;
the converged H is the unique root of N(H) = N_res, so the two agree to
about 1.5x the stopping tolerance (bar: 1e-6 relative)."""
import numpy as np
import pytest
import torch

import crk_inputs as ci
import oracle
from paper_2202_02840_amd import CRK_FP64, Context, CrkError
from paper_2202_02840_amd import pipeline as pl

pytestmark = pytest.mark.gpu


def _gpu_hsolve(ps, nres, tol=1e-7, max_iter=100, start=None, tune=None):
    ctx = Context(0)
    if tune:
        ctx.set_hsolve(*tune)
    dev = pl.upload(ps)
    H0 = dev["H"] if start is None else torch.as_tensor(start, device="cuda")
    prm = pl.params_for(ps, nres, CRK_FP64)
    ctx.build_cells(dev["x"], dev["y"], dev["z"], H0, prm)
    Hs = ctx.permute(H0.contiguous(), True)
    Hn, it, nun = ctx.hsolve(nres, Hs, tol, max_iter)
    torch.cuda.synchronize()
    H = ctx.permute(Hn, False).cpu().numpy()
    perm = ctx.perm.long().cpu().numpy()
    iters = np.empty(ps.n, dtype=np.int32)
    iters[perm] = it.cpu().numpy()
    return H, iters, nun, ctx


@pytest.mark.parametrize("name,make", [
    ("lognormal16", lambda: ci.lognormal_box(16, sigma=1.5, seed=301)),
    ("lattice12", lambda: ci.lattice_box(12, seed=302)),
])
@pytest.mark.parametrize("tune", [None, (4, 8, -1, 0.0), (2, 3, 8, 0.0), (16, 8, 320, 1.05)],
                         ids=["rows", "no-rows", "overflow", "tight-rows"])
def test_hsolve_matches_oracle(name, make, tune):
    ps = make()
    print(f"[case] hsolve {name} tune={tune} n={ps.n}", flush=True)
    # sparse particles, where N(H) is flat, contract slowly: allow 1000 updates
    Href, itref, nf = oracle.hsolve(ps.x, ps.y, ps.z, ps.H, 64.0, tol=1e-7, max_iter=1000)
    H, it, nun, _ = _gpu_hsolve(ps, 64.0, max_iter=1000, tune=tune)
    assert nf == 0 and nun == 0
    assert np.abs(H / Href - 1).max() < 1e-6
    # same update on both sides: iteration counts agree up to the last step
    assert np.abs(it - itref).max() <= 1


def test_hsolve_narrow_and_wide_passes_match_oracle():
    """A clustered set large enough that the iteration starts with 8 lanes per
    particle: particles whose candidate row overflows are handed to the wide
    pass (a wavefront per particle, pool rows) and back; with a short row
    (cap 96) most of them go through it. Register rows (16 and 8 lanes, one
    launch for both passes) and memory rows (32 lanes, two launches) all
    match the oracle."""
    ps = ci.lognormal_box(48, sigma=2.0, seed=305)
    print(f"[case] hsolve narrow/wide n={ps.n}", flush=True)
    Href, itref, nf = oracle.hsolve(ps.x, ps.y, ps.z, ps.H, 64.0, tol=1e-7, max_iter=1000)
    assert nf == 0
    for tune in (None, (8, 8, 96, 1.3), (32, 8, 320, 1.3)):
        H, it, nun, _ = _gpu_hsolve(ps, 64.0, max_iter=1000, tune=tune)
        print(tune, "max rel", float(np.abs(H / Href - 1).max()), flush=True)
        assert nun == 0
        assert np.abs(H / Href - 1).max() < 1e-6
        assert np.abs(it - itref).max() <= 1


def test_update_support_rebuilds_lists():
    """After crk_update_support with new support radii (the oracle's converged
    H), the pair lists equal the oracle's for those radii."""
    ps = ci.lognormal_box(14, sigma=1.5, seed=303)
    print(f"[case] update_support n={ps.n}", flush=True)
    Hc, _, _ = oracle.hsolve(ps.x, ps.y, ps.z, ps.H, 64.0, tol=1e-7, max_iter=1000)
    ctx = Context(0)
    dev = pl.upload(ps)
    ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], pl.params_for(ps, 64.0, CRK_FP64))
    Hs = ctx.permute(torch.as_tensor(Hc, device="cuda"), True)
    npairs = ctx.update_support(Hs)
    soff, sidx = oracle.neighbors(ps.x, ps.y, ps.z, Hc, 1.0, True, 1)
    assert npairs == soff[-1]
    from gpu_helpers import rows_original
    off, idx = ctx.export_neighbors(1)
    rows = rows_original(off, idx, ctx.perm)
    for i in range(ps.n):
        assert np.array_equal(rows[i], sidx[soff[i]:soff[i + 1]]), i


def test_hsolve_rejects_target_below_self_term():
    ps = ci.lattice_box(8, seed=304)
    print(f"[case] hsolve bad Nres n={ps.n}", flush=True)
    with pytest.raises(CrkError):
        _gpu_hsolve(ps, 20.0)
