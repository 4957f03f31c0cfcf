"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs, element by element.

Bars: neighbour sets bit-exact; FP64 path within 1e-12 normwise relative
error per output; mixed path (FP32 pair terms, Kahan sums, FP64 solve)
within 1e-5. Sizes span several 256-thread tiles with ragged tails."""
import numpy as np
import pytest

import crk_inputs as ci
import oracle
from gpu_helpers import OUTPUTS, compare, gpu_run, oracle_run, rows_original
from paper_2202_02840_amd import CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT, Context

pytestmark = pytest.mark.gpu

CASES = {
    "lattice16": lambda: ci.lattice_box(16, seed=101),
    "lognormal20": lambda: ci.lognormal_box(20, sigma=1.5, seed=102),
    "lognormal_ragged": lambda: ci.lognormal_box(17, sigma=1.5, seed=103),   # 4913 particles
}


def _print_case(name, ps):
    print(f"[case] {name} n={ps.n}", flush=True)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("walk", [(4, 192, 0), (1, 192, 0), (8, 16, 0), (16, 3, 0), (4, 192, 1), (8, 16, 2)])
def test_neighbour_lists_bit_exact(name, which, walk):
    ps = CASES[name]()
    _print_case(f"{name} walk {walk}", ps)
    res = gpu_run(ps, walk=walk)
    ctx = res["ctx"]
    off, idx = ctx.export_neighbors(which)
    rows = rows_original(off, idx, ctx.perm)
    ooff, oidx = oracle.neighbors(ps.x, ps.y, ps.z, ps.H, ps.L, True, which)
    for i in range(ps.n):
        assert np.array_equal(rows[i], oidx[ooff[i]:ooff[i + 1]]), i
    if which == 1:
        assert res["n_pairs"] == ooff[-1]


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_path_matches_oracle(name):
    ps = CASES[name]()
    _print_case(name, ps)
    ref = oracle_run(ps)
    res = gpu_run(ps, CRK_FP64)
    assert res["n_singular"] == ref["n_singular"]
    errs = compare(res, ref)
    print(errs)
    for k, e in errs.items():
        assert e <= 1e-12, (k, e)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [CRK_MIXED, CRK_MIXED_ADAPT])
def test_mixed_path_matches_oracle(name, prec):
    ps = CASES[name]()
    _print_case(name, ps)
    ref = oracle_run(ps)
    res = gpu_run(ps, prec)
    errs = compare(res, ref)
    print(errs)
    for k, e in errs.items():
        assert e <= 1e-5, (k, e)


@pytest.mark.parametrize("lanes", [(1, 1, 1, 1), (2, 2, 2, 2), (16, 4, 16, 16), (64, 8, 32, 64)])
def test_every_lane_split_agrees(lanes):
    ps = CASES["lognormal_ragged"]()
    _print_case(f"lanes {lanes}", ps)
    ref = oracle_run(ps)
    for prec, tol in ((CRK_FP64, 1e-12), (CRK_MIXED, 1e-5), (CRK_MIXED_ADAPT, 1e-5)):
        res = gpu_run(ps, prec, lanes=lanes)
        errs = compare(res, ref)
        for k, e in errs.items():
            assert e <= tol, (prec, lanes, k, e)


def test_bitwise_deterministic():
    ps = CASES["lognormal20"]()
    _print_case("determinism", ps)
    a = gpu_run(ps, CRK_MIXED)
    b = gpu_run(ps, CRK_MIXED)
    for k in OUTPUTS:
        assert np.array_equal(a[k], b[k]), k


def test_adaptive_mode_with_every_row_fp64_equals_fp64_path():
    """kappa_max = 0 sends every row through the FP64 launches: the result then
    matches the FP64 path to rounding."""
    ps = CASES["lognormal20"]()
    _print_case("adaptive kappa 0", ps)
    a = gpu_run(ps, CRK_FP64)
    b = gpu_run(ps, CRK_MIXED_ADAPT, kappa_max=0.0)
    assert b["ctx"].adaptive_rows()[0] == ps.n
    for k in OUTPUTS:
        den = np.abs(a[k]).max()
        assert np.abs(a[k] - b[k]).max() <= 1e-13 * max(den, 1e-300), k


def test_paper_resolution_nres_268():
    """The paper's resolution, N_res = 268 (n_h = 4): a clustered box with H
    sized for 268 neighbours (rows past the walk's scratch cap take the long
    path), lists bit-exact, FP64 path within 1e-12, adaptive within 1e-5."""
    ps = ci.lognormal_box(24, sigma=1.5, seed=941, nngb=268.0, hcap=0.45)
    _print_case("lognormal 24^3 N_res 268", ps)
    ref = oracle_run(ps, nres=268.0)
    assert ref["n_pairs"] / ps.n > 250
    for prec, tol in ((CRK_FP64, 1e-12), (CRK_MIXED_ADAPT, 1e-5)):
        res = gpu_run(ps, prec, nres=268.0)
        ctx = res["ctx"]
        off, idx = ctx.export_neighbors(1)
        rows = rows_original(off, idx, ctx.perm)
        for i in range(0, ps.n, 97):
            assert np.array_equal(rows[i], ref["sidx"][ref["soff"][i]:ref["soff"][i + 1]]), i
        assert res["n_pairs"] == ref["n_pairs"]
        errs = compare(res, ref)
        print(prec, {k: f"{e:.1e}" for k, e in errs.items()})
        for k, e in errs.items():
            assert e <= tol, (prec, k, e)


def test_walk_cap_grows_after_long_rows():
    """Supports for 268 neighbours overflow the default 192-slot walk rows,
    so the first build walks nearly every row twice; the next build on the
    same context sizes its scratch rows from the first one's mean and longest
    rows (more workspace) and gives the same lists and the same sums bit for
    bit."""
    ps = ci.lognormal_box(24, sigma=1.5, seed=941, nngb=268.0, hcap=0.45)
    _print_case("lognormal 24^3 N_res 268, two builds", ps)
    ref = oracle_run(ps, nres=268.0)
    ctx = Context(0)
    outs, held = [], []
    for _ in range(2):
        res = gpu_run(ps, CRK_FP64, nres=268.0, ctx=ctx)
        held.append(ctx.workspace_bytes())
        off, idx = ctx.export_neighbors(1)
        rows = rows_original(off, idx, ctx.perm)
        for i in range(ps.n):
            assert np.array_equal(rows[i], ref["sidx"][ref["soff"][i]:ref["soff"][i + 1]]), i
        assert res["n_pairs"] == ref["n_pairs"]
        outs.append({k: np.array(res[k]) for k in OUTPUTS})
    assert held[1] > held[0]
    for k in OUTPUTS:
        assert np.array_equal(outs[0][k], outs[1][k]), k
