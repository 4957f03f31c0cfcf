"""Throughput of the CRKSPH step on one MI355X.

Workload: 128^3 = 2,097,152 gas particles, lognormal clustered positions
(sigma_ln rho = 1.5, P(k) ~ k^-2 on a 128^3 grid, seed 2), H sized for 64
neighbours at each particle's cell density (neighbour counts ~20-400), gas
state u = 1, masses 1/N, density m/V, shear + noise velocities. One step is
every pass of the hot path: cell sort + neighbour lists, volumes, kernel
moments, FP64 RK solve, velocity gradient, momentum/energy derivatives with
limited viscosity, in the mixed precision (FP32 pair terms with Kahan sums,
FP64 solve) unless --precision fp64.

Prints one JSON line: pair-interactions/s (ordered pairs (i, j), j in N_s(i),
counted once per step) over the whole step, the per-kernel roofline of the
derivative pass, the max normwise error of every output against the FP64
GPU path, and the FP64 CPU oracle timed on a smaller box of the same recipe.
Further legs: the same step recorded once as a HIP graph and replayed
(graph_replay), the smoothing-length network against the plain iteration
(h_surrogate), 512 independent boxes of 8^3..48^3 particles in one
batched, graph-recorded step (batch), and one complete step of the
256^3 clumped set with its smoothing-length iteration (full_size).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks: HBM3E bandwidth, and the vector ALU rate of code compiled
# without packed FP32 instructions (as the library is).
# 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s for
# FP64 and for unpacked FP32; the 157.3 TFLOP/s FP32 figure needs packed
# FP32 instructions, which this library is compiled without.
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 78.6
VALU_PEAK_PACKED_FP32 = 157.3

# algorithmic work of the derivative pass (k_deriv), counted from the kernel
# source (pair_deriv in crk_pairs.hip, an FMA counted as two flops, sqrt,
# reciprocal and exp as one, the separation d not counted): 187 flops per
# ordered pair, 4 of them the sums; bytes per particle: the packed record
# (FP32: 144 bytes, the position riding in its padding as 42-bit fixed
# point; FP64: 256 of 288, plus x, y, z (24)), m (8), row offsets (16),
# outputs (32); per ordered pair its 4-byte index
DERIV_FLOPS_PER_PAIR = 187
DERIV_BYTES_PER_PARTICLE = {"mixed": 144 + 8 + 16 + 32, "fp64": 24 + 256 + 8 + 16 + 32}
DERIV_BYTES_PER_PAIR = 4

OUT_KEYS = ("V", "m0", "m1", "m2", "gm0", "gm1", "gm2", "A", "B", "gA", "gB", "gradv", "dpdt",
            "dudt")


COUNTERS = os.path.join(ROOT, "profiles", "k_deriv_counters.json")
# steps after the timed region whose every kernel is timed (the breakdown)
BREAKDOWN_STEPS = 10
DERIV_SOURCE = os.path.join(ROOT, "paper_2202_02840_amd", "csrc", "crk_pairs.hip")


def code_sha256(path: str) -> str:
    """Hash of a C++ source with its comments and blank lines removed, so a
    change of comments alone does not count as a change of the kernel."""
    import hashlib
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    lines = [ln.rstrip() for ln in src.splitlines() if ln.strip()]
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def deriv_traffic(precision: str, lanes: int):
    """HBM bytes per k_deriv launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by the copy-probe factors), or None when
    the kernel source (its code, comments aside) or its launch shape (the
    particles per wavefront of its balanced lane groups) differs from the
    one measured."""
    if not os.path.exists(COUNTERS):
        return None
    rec = json.load(open(COUNTERS))
    if (rec.get("source_code_sha256") != code_sha256(DERIV_SOURCE) or
            rec.get("precision") != precision or rec.get("lanes") != lanes):
        return None
    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0


def make_workload(n_side=128, seed=2):
    import crk_inputs as ci
    return ci.lognormal_box(n_side, sigma=1.5, spectral_index=-2.0, seed=seed)


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_step_rate(ps) -> tuple:
    """(pairs, seconds) of the oracle's whole step on one particle set."""
    import oracle
    t0 = time.perf_counter()
    out = oracle.pipeline(ps, oracle.params(64.0, gamma=ps.gamma))
    return int(out["n_pairs"]), time.perf_counter() - t0


def cpu_baseline(n_side: int) -> dict:
    import oracle
    ps = make_workload(n_side)
    prm = oracle.params(64.0)
    t0 = time.perf_counter()
    out = oracle.pipeline(ps, prm)
    dt = time.perf_counter() - t0
    res = {"value": out["n_pairs"] / dt, "unit": "pair-interactions/s", "cores": oracle.threads(),
           "cpu_model": cpu_model(), "kind": "oracle",
           "sample": f"full FP64 oracle step (neighbour sets, volume, moments, corrections, grad v, "
                     f"derivatives) on the same recipe at {n_side}^3 = {ps.n} particles "
                     f"({out['n_pairs']} pairs, {dt:.2f} s)"}
    # the oracle's compatible energy pass on the same state, beside the GPU's
    t0 = time.perf_counter()
    oracle.compatible_energy(ps.x, ps.y, ps.z, ps.H, ps.v, ps.m, ps.u, ps.rho, out["V"], out,
                             out["gradv"], out["soff"], out["sidx"], prm, out["dvdt"], 1e-3, ps.L)
    dtc = time.perf_counter() - t0
    res["compatible_energy"] = {"value": out["n_pairs"] / dtc, "cores": oracle.threads(),
                                "sample": f"the oracle's compatible pass at {n_side}^3 "
                                          f"({out['n_pairs']} pairs, {dtc:.2f} s)"}
    # the same oracle on one host thread, in a child process (its OpenMP
    # team size is fixed when the library loads), on a 32^3 sample
    import subprocess
    code = ("import json, sys, time; sys.path.insert(0, %r); import bench, oracle; "
            "ps = bench.make_workload(32); t = time.perf_counter(); "
            "o = oracle.pipeline(ps, oracle.params(64.0)); d = time.perf_counter() - t; "
            "print(json.dumps({'pairs': int(o['n_pairs']), 'seconds': d, 'threads': oracle.threads()}))"
            % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300, check=True)
        one = json.loads(r.stdout.strip().splitlines()[-1])
        res["one_thread"] = {"value": one["pairs"] / one["seconds"], "cores": one["threads"],
                             "sample": f"the same oracle step at 32^3 ({one['pairs']} pairs, "
                                       f"{one['seconds']:.2f} s)"}
    except (subprocess.SubprocessError, ValueError, KeyError, IndexError) as e:
        res["one_thread"] = {"error": str(e)[:200]}
    # the oracle on the other configurations: the 32^3 jittered lattice whole,
    # and a sample of the 512-box batch (every 16th box)
    import crk_inputs as ci
    from paper_2202_02840_amd import pipeline as pl
    c1 = ci.lattice_box(32, seed=1)
    pr, sec = oracle_step_rate(c1)
    res["c1_lattice_32"] = {"value": pr / sec, "cores": oracle.threads(),
                            "sample": f"whole oracle step, 32^3 jittered lattice ({pr} pairs, {sec:.2f} s)"}
    boxes = ci.batch_boxes(512, seed=3)[::16]
    pr, sec = 0, 0.0
    for b in boxes:
        p1, s1 = oracle_step_rate(b)
        pr += p1
        sec += s1
    res["c3_batch_sample"] = {"value": pr / sec, "cores": oracle.threads(),
                              "sample": f"whole oracle step on every 16th of the 512 boxes "
                                        f"({len(boxes)} boxes, {sum(b.n for b in boxes)} particles, "
                                        f"{pr} pairs, {sec:.2f} s)"}
    return res


def hsurrogate_leg(ctx, args) -> dict:
    """Smoothing-length network: labels from the plain iteration on clustered
    boxes of 64^3..128^3 (sigma_ln_rho drawn from U[1, 2]), each box twice:
    cold (the generator's supports, sized from the smoothed grid density)
    and warm (the converged supports carried over a Courant step of
    motion); training with the library's own kernels; then, on a held-out
    128^3 box (sigma 2.0) from a cold and from a warm start, the plain
    iteration against the network-seeded one at identical converged H, with
    the tail of the per-particle update counts."""
    import crk_inputs as ci
    import torch
    from paper_2202_02840_amd import hsurrogate as hs
    t0 = time.perf_counter()
    feats, tgts, nsamp, boxes = [], [], 0, []
    rng = np.random.default_rng(100)
    sides = [int(v) for v in args.hs_train_sides.split(",")]
    sigmas = rng.uniform(1.0, 2.0, size=len(sides))
    for b, (side, sg) in enumerate(zip(sides, sigmas)):
        ps = ci.lognormal_box(side, sigma=float(sg), seed=100 + b)
        for start in ("cold", "warm"):
            src = ps if start == "cold" else hs.moved(ps, hs.converged(ctx, ps))
            f, t, _ = hs.training_pairs(ctx, src)
            feats.append(f)
            tgts.append(t)
            nsamp += src.n
        boxes.append(f"{side}^3 sigma {sg:.2f}")
    t1 = time.perf_counter()
    theta, hist = hs.train(ctx, ci.hnet_init(0), feats, tgts, steps=args.hs_steps, batch=8192,
                           log_every=max(args.hs_steps // 5, 1))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del feats, tgts
    held = ci.lognormal_box(args.hs_eval_side, sigma=2.0, seed=4)
    r = {"cold": hs.evaluate(ctx, held, theta, tol=1e-8, repeats=2)}
    r["warm"] = hs.evaluate(ctx, hs.moved(held, hs.converged(ctx, held)), theta, tol=1e-8, repeats=2)
    r.update(speedup=r["cold"]["speedup"], max_rel_dH=max(r["cold"]["max_rel_dH"], r["warm"]["max_rel_dH"]),
             train_samples=nsamp, train_boxes=boxes, train_starts="cold and warm per box",
             train_steps=args.hs_steps, label_seconds=t1 - t0, train_seconds=t2 - t1,
             loss_history=hist, eval_box=f"lognormal {args.hs_eval_side}^3, sigma 2.0, seed 4")
    return r, theta


def full_size_leg(args, prec, theta=None) -> dict:
    """The largest single-GPU set: 256^3 particles, lognormal (sigma 2.0,
    P(k) ~ k^-2.5) with 1% of them in 64 dense clumps (seed 5). One complete
    step: the smoothing-length iteration from the generator's supports
    (plain, and seeded by the trained network when one is given), then the
    build and every pass at the converged supports; mixed against the FP64
    GPU path."""
    import crk_inputs as ci
    import torch
    from paper_2202_02840_amd import CRK_FP64, Context
    from paper_2202_02840_amd import autotune as at
    from paper_2202_02840_amd import pipeline as pl
    t0 = time.perf_counter()
    ps = ci.clustered_clump_box(args.full_side)
    gen_s = time.perf_counter() - t0
    ctx = Context(0)
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, prec, kappa_max=args.kappa)
    ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], prm)
    Hs = ctx.permute(dev["H"], True)
    hres = {}
    for name in ("plain", "surrogate"):
        if name == "surrogate" and theta is None:
            continue
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        start = Hs if name == "plain" else ctx.hnet_seed(theta, 64.0, Hs)
        Hc, it, nun = ctx.hsolve(64.0, start, 1e-8, 1000)
        torch.cuda.synchronize()
        hres[name] = dict(seconds=time.perf_counter() - t1, mean_iters=float(it.double().mean()),
                          max_iters=int(it.max()), unconverged=int(nun), H=Hc)
        ctx.update_support(Hs)
    use = "surrogate" if "surrogate" in hres else "plain"
    Hconv = hres[use]["H"]
    if "surrogate" in hres:
        hres["max_rel_dH"] = float((hres["surrogate"]["H"] / hres["plain"]["H"] - 1).abs().max())
        hres["speedup"] = hres["plain"]["seconds"] / hres["surrogate"]["seconds"]
    # the converged supports in the original order
    dev["H"] = ctx.permute(Hconv, False)
    for k in ("plain", "surrogate"):
        if k in hres:
            hres[k].pop("H")
    out = pl.step(ctx, dev, prm, count_singular=False)
    cfg = at.load(prec, out["n_pairs"] / ps.n)
    if cfg:
        at.apply(ctx, cfg)
    for _ in range(args.warmup):
        out = pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        out = pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t2) * 1e3 / max(args.steps, 1)
    npairs = int(out["n_pairs"])
    # per-kernel event times from two more steps (every kernel bracketed)
    ctx.timing(True)
    ctx.timing_reset()
    for _ in range(2):
        pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    kern = {}
    for k in ("sort", "k_walk", "k_compact_rows", "k_walk_long", "k_extra_rank", "k_volume", "k_moments",
              "k_corrections", "k_flag", "k_pack", "k_gradv", "k_gradv_fix", "k_deriv", "k_deriv_fix"):
        kms, cnt = ctx.timing_read(k)
        kern[k] = kms / max(cnt, 1)
    ctx.timing(False)
    res = {"workload": f"lognormal {args.full_side}^3 sigma 2.0, P(k)~k^-2.5, 1% in 64 clumps at "
                       f"100x mean density, seed 5; h iteration from the generator's H to 1e-8, "
                       f"then the {args.precision} step at the converged H",
           "particles": ps.n, "pairs_per_step": npairs, "step_ms": ms,
           "step_pairs_per_s": npairs / (ms * 1e-3), "h_iteration": hres,
           "h_iteration_used": use,
           "full_step_ms": ms + hres[use]["seconds"] * 1e3, "lanes": cfg, "kernel_ms": kern,
           "generate_seconds": gen_s}
    if not args.no_check:
        ref = pl.step(ctx, dev, pl.params_for(ps, 64.0, CRK_FP64), count_singular=False)
        cur = pl.step(ctx, dev, prm, count_singular=False)
        torch.cuda.synchronize()
        errs = {}
        for k in OUT_KEYS:
            a, b = cur[k], ref[k]
            den = b.abs().max().item()
            errs[k] = (a - b).abs().max().item() / den if den > 0 else (a - b).abs().max().item()
        res["max_rel_err_vs_fp64"] = errs
        res["err_target_met"] = bool(max(errs.values()) <= 1e-5)
    return res


def timestep_leg(ctx, dev, prm, args) -> dict:
    """The Courant terms of Sec. 3.1 fused into the derivative pass: the same
    step with the terms on, the derivative pass's event time against the
    plain one (alternating blocks of steps with and without, events on the
    derivative pass only), and the per-particle combination (crk_timestep)."""
    import torch
    from paper_2202_02840_amd import pipeline as pl
    for _ in range(max(args.warmup, 1)):
        pl.step(ctx, dev, prm, count_singular=False, timestep=True)
    torch.cuda.synchronize()

    def block(ts):
        ctx.timing(True)
        ctx.timing_only("k_deriv")
        ctx.timing_reset()
        for _ in range(args.steps):
            o = pl.step(ctx, dev, prm, count_singular=False, timestep=ts)
        torch.cuda.synchronize()
        ms, cnt = ctx.timing_read("k_deriv")
        ctx.timing_only(None)
        ctx.timing(False)
        return ms / max(cnt, 1), o

    with_ts, plain = [], []
    for _ in range(2):
        t, out = block(True)
        with_ts.append(t)
        plain.append(block(False)[0])
    der, deriv_ms_plain = float(np.mean(with_ts)), float(np.mean(plain))
    vmax, dt = out["vmax"], out["dt_hyd"]
    return {"k_deriv_ms": der, "k_deriv_ms_without": deriv_ms_plain,
            "overhead": der / deriv_ms_plain - 1.0,
            "vmax_range": [float(vmax.min()), float(vmax.max())],
            "dt_hyd_range": [float(dt.min()), float(dt.max())],
            "terms": "v_sig, c_sq (zeta 4), c_s, h_hat |div u| / a; dt_hyd = 0.25 h_hat / v_max"}


def compat_leg(ctx, dev, prm, args, deriv_ms_plain: float, dt: float = 1e-3) -> dict:
    """The compatible energy update over a step dt (a second pair pass that
    recomputes each pair's dp_ij/dt): its event time, its energy balance on
    the whole workload (the thermal energy the pairs hand out against the
    kinetic change, which cancel exactly for the method), and its error
    against the FP64 path of the same pass on the same state."""
    import torch
    from paper_2202_02840_amd import CRK_FP64
    from paper_2202_02840_amd import pipeline as pl
    for _ in range(max(args.warmup, 1)):
        pl.step(ctx, dev, prm, count_singular=False, compat_dt=dt)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_reset()
    for _ in range(args.steps):
        out = pl.step(ctx, dev, prm, count_singular=False, compat_dt=dt)
    torch.cuda.synchronize()
    ms, cnt = ctx.timing_read("k_compat")
    fms, fcnt = ctx.timing_read("k_compat_fix")
    ctx.timing(False)
    perm = out["perm"].long()
    m = dev["m"].index_select(0, perm)
    u = dev["u"].index_select(0, perm)
    v = dev["v"].index_select(1, perm)
    a = prm.a
    p0 = a * v
    p1 = p0 + dt * out["dpdt"]
    dkin = (m * ((p1 * p1).sum(0) - (p0 * p0).sum(0))).sum() / (2.0 * a ** 4)
    pair = m * (out["du_compat"] + dt * (prm.adot / a) * (3.0 * (prm.gamma - 1.0) + 2.0) * u)
    balance = (pair.sum() + dkin).abs().item() / pair.abs().sum().item()
    res = {"dt": dt, "k_compat_ms": ms / max(cnt, 1),
           "k_compat_fix_ms": fms / max(fcnt, 1) if fcnt else 0.0,
           "k_deriv_ms": deriv_ms_plain,
           "energy_balance_rel": balance}
    if not args.no_check:
        p64 = type(prm).from_buffer_copy(prm)
        p64.precision = CRK_FP64
        from paper_2202_02840_amd import Context
        ref = pl.step(Context(0), dev, p64, count_singular=False, compat_dt=dt)
        torch.cuda.synchronize()
        a_ = out["du_compat"]
        b_ = ref["du_compat"]
        res["max_rel_err_vs_fp64"] = (a_ - b_).abs().max().item() / b_.abs().max().item()
    return res


def verlet_leg(ctx, args, prec) -> dict:
    """Velocity-Verlet hydro steps (eq. verletOP), each the half kicks and
    drift around one whole evaluation at the predicted state, on a jittered
    lattice of the same particle count (uniform gas in a gentle shear flow;
    the clustered workload starts far from pressure balance, and the energy
    derivative of eq. eng, which weights each pair by the partner's
    pressure, drives its thinnest particles to negative energy within a few
    Courant steps). Reports the wall time per step, the elementwise kernels'
    share and the change of the total energy sum m (u + |p|^2 / (2 a^4)).
    The step is the smallest Courant step dt_hyd of the start state
    (Sec. 3.1, C_CFL = 0.25)."""
    import torch
    import crk_inputs as ci
    from paper_2202_02840_amd import pipeline as pl
    ps = ci.lattice_box(args.n_side, seed=6, vamp=0.1)
    ps.rho = None
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, prec)
    dt = float(pl.step(ctx, dev, prm, count_singular=False, timestep=True)["dt_hyd"].min())
    n = ps.n
    st = {k: (v.clone() if v is not None else None) for k, v in dev.items()}
    st["dpdt"] = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    st["dudt"] = torch.zeros(n, dtype=torch.float64, device="cuda")
    a = prm.a

    def energy():
        return (st["m"] * (st["u"] + (a * st["v"]).pow(2).sum(0) / (2.0 * a ** 4))).sum().item()

    res = {"workload": f"jittered lattice {args.n_side}^3, uniform gas, shear flow v_x = 0.1 sin(2 pi y), seed 6",
           "dt": dt, "steps": args.steps}
    for mode in ("eng", "compat"):
        for k in ("x", "y", "z", "v", "u"):
            st[k].copy_(dev[k])
        ctx.verlet_step(st, prm, dt, start_eval=True, energy=mode)
        e0 = energy()
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_reset()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.verlet_step(st, prm, dt, energy=mode)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
        vms, _ = ctx.timing_read("k_verlet")
        cms, _ = ctx.timing_read("k_compat")
        ctx.timing(False)
        res[mode] = {"ms_per_step": ms, "k_verlet_ms_per_step": vms / max(args.steps, 1),
                     "k_compat_ms_per_step": cms / max(args.steps, 1),
                     "energy_rel_change": abs(energy() - e0) / abs(e0)}
    return res


def nres268_leg(args, prec) -> dict:
    """Sensitivity point at the paper's resolution, N_res = 268 (n_h = 4,
    Sec. 3.6): the same clustered 128^3 recipe with H sized for 268
    neighbours, the whole step timed, the derivative pass's roofline, and
    the error against the FP64 GPU path. Lanes from the stored table for
    this pair density (the nearest entry)."""
    import torch
    import crk_inputs as ci
    from paper_2202_02840_amd import CRK_FP64, Context
    from paper_2202_02840_amd import autotune as at
    from paper_2202_02840_amd import pipeline as pl
    ps = ci.lognormal_box(args.n_side, sigma=1.5, spectral_index=-2.0, seed=2, nngb=268.0)
    dev = pl.upload(ps)
    ctx = Context(0)
    prm = pl.params_for(ps, 268.0, prec, kappa_max=args.kappa)
    first = pl.step(ctx, dev, prm, count_singular=False)
    tuned = at.load(prec, first["n_pairs"] / ps.n)
    if tuned:
        at.apply(ctx, tuned)
    for _ in range(max(args.warmup, 1)):
        out = pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_reset()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    dms, dcnt = ctx.timing_read("k_deriv")
    ctx.timing(False)
    npairs = int(out["n_pairs"])
    t_der = dms / max(dcnt, 1) * 1e-3
    tf = DERIV_FLOPS_PER_PAIR * npairs / t_der / 1e12
    res = {"workload": f"lognormal clustered gas, {args.n_side}^3, sigma_ln_rho 1.5, P(k)~k^-2, "
                       f"268-neighbour H, seed 2; N_res = 268",
           "pairs_per_step": npairs, "mean_pairs_per_particle": npairs / ps.n,
           "ms_per_step": ms, "pairs_per_s": npairs / (ms * 1e-3),
           "k_deriv_ms": t_der * 1e3, "k_deriv_tflops": tf, "k_deriv_frac": tf / VALU_PEAK_TFLOPS,
           "lanes": tuned}
    if not args.no_check:
        ref = pl.step(ctx, dev, pl.params_for(ps, 268.0, CRK_FP64), count_singular=False)
        cur = pl.step(ctx, dev, prm, count_singular=False)
        torch.cuda.synchronize()
        res["max_rel_err_vs_fp64"] = max(
            (cur[k] - ref[k]).abs().max().item() / max(ref[k].abs().max().item(), 1e-300)
            for k in OUT_KEYS)
    del ctx, dev
    torch.cuda.empty_cache()
    return res


def wave_balance(row_len, per_wave: int) -> dict:
    """Load balance of the derivative pass over the sorted order: pairs per
    wavefront of `per_wave` consecutive particles (mean, coefficient of
    variation, max / mean), and the lane efficiency of two mappings: G = 8
    lanes per particle (a wave runs as long as its longest row) and the
    balanced lane groups (lanes split by row length, one plus a share of
    the rest each)."""
    import numpy as np
    n = len(row_len)
    m = (n // per_wave) * per_wave
    L = np.asarray(row_len[:m], dtype=np.int64).reshape(-1, per_wave)
    w = L.sum(axis=1).astype(np.float64)
    steps_g8 = np.ceil(L / 8.0).max(axis=1)
    eff_g8 = L.sum() / (64.0 * steps_g8.sum())
    # balanced groups: p gets 1 + floor((64 - P) * prefix / S) lanes (prefix differences)
    S = np.maximum(L.sum(axis=1, keepdims=True), 1)
    pre = np.concatenate([np.zeros((L.shape[0], 1), np.int64), np.cumsum(L, axis=1)], axis=1)
    start = np.arange(per_wave + 1)[None, :] + ((64 - per_wave) * pre) // S
    start[:, -1] = 64
    g = np.diff(start, axis=1)
    steps_bal = np.ceil(L / np.maximum(g, 1)).max(axis=1)
    eff_bal = L.sum() / (64.0 * steps_bal.sum())
    return {"particles_per_wave": per_wave, "pairs_per_wave_mean": float(w.mean()),
            "pairs_per_wave_cv": float(w.std() / w.mean()), "pairs_per_wave_max_over_mean":
            float(w.max() / w.mean()), "lane_efficiency_g8": float(eff_g8),
            "lane_efficiency_balanced": float(eff_bal)}


def leaves_leg(args, prec, n_side: int, sigma: float, spectral: float, seed: int, clumps: bool,
               label: str) -> dict:
    """RCB leaf tiling (Sec. 3.3) against the Morton cell build on one
    clustered box: build times, the pair passes on the lists of each (in
    each one's sorted order), the load balance of the derivative pass over
    waves, and the leaf statistics (sizes, partners per leaf)."""
    import numpy as np
    import torch
    import crk_inputs as ci
    from paper_2202_02840_amd import Context
    from paper_2202_02840_amd import autotune as at
    from paper_2202_02840_amd import pipeline as pl
    if clumps:
        ps = ci.clustered_clump_box(n_side, sigma=sigma, spectral_index=spectral, seed=seed)
    else:
        ps = ci.lognormal_box(n_side, sigma=sigma, spectral_index=spectral, seed=seed)
    dev = pl.upload(ps)
    ctx = Context(0)
    prm = pl.params_for(ps, 64.0, prec, kappa_max=args.kappa)
    first = pl.step(ctx, dev, prm, count_singular=False)
    tuned = at.load(prec, first["n_pairs"] / ps.n)
    if tuned:
        at.apply(ctx, tuned)
    out = {"workload": label, "particles": ps.n}
    passes = ("k_volume", "k_moments", "k_corrections", "k_gradv", "k_deriv", "k_deriv_fix")

    def run(kind):
        rec = {}
        ts = []
        for rep in range(max(args.warmup, 1) + 3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "morton":
                perm, npairs = ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], prm)
            else:
                perm, npairs, loff = ctx.build_leaves(dev["x"], dev["y"], dev["z"], dev["H"], prm,
                                                      256, 32)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        rec["build_ms_median_of_3"] = float(np.median(ts[-3:]) * 1e3)
        rec["pairs"] = int(npairs)
        v = ctx.permute(dev["v"], True)
        m = ctx.permute(dev["m"], True)
        u = ctx.permute(dev["u"], True)
        ctx.timing(True)
        ctx.timing_reset()
        for _ in range(3):
            mom = ctx.moments(prm)
            corr = ctx.corrections(mom, count_singular=False)
            ctx.derivatives(prm, v, m, u, None, mom["V"], corr)
        torch.cuda.synchronize()
        rec["kernel_ms"] = {k: ctx.timing_read(k)[0] / max(ctx.timing_read(k)[1], 1) for k in passes}
        ctx.timing(False)
        off, _ = ctx.export_neighbors(1)
        lens = np.diff(off.cpu().numpy())
        rec["balance"] = wave_balance(lens, 8)
        if kind == "rcb":
            lo = loff.cpu().numpy()
            sz = np.diff(lo)
            rec["leaves"] = int(len(sz))
            rec["leaf_size_min_max"] = [int(sz.min()), int(sz.max())]
        return rec

    out["morton"] = run("morton")
    out["rcb"] = run("rcb")
    out["rcb"]["leaf_pairs_per_leaf"] = None
    assert out["morton"]["pairs"] == out["rcb"]["pairs"], "the two tilings must give the same N_s"
    del ctx, dev
    torch.cuda.empty_cache()
    return out


def graph_replay_ms(ctx, io, prm, steps: int, warmup: int, box_offsets=None) -> tuple:
    """Record the step as one HIP graph on the buffers of io and time its
    replays (synchronised wall clock); returns (ms per replay, status)."""
    import torch
    ctx.graph_capture(io, prm, box_offsets=box_offsets, headroom=0.25)
    for _ in range(warmup):
        ctx.graph_replay(status=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.graph_replay(status=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    st, info = ctx.graph_replay()
    return ms, st, info


def batch_leg(args, prec, precision_name: str) -> dict:
    """Many independent boxes of uneven size in one build and one launch per
    pass, the whole step recorded once as a HIP graph and replayed."""
    import crk_inputs as ci
    import torch
    from paper_2202_02840_amd import CRK_FP64, Context
    from paper_2202_02840_amd import autotune as at
    from paper_2202_02840_amd import pipeline as pl
    t0 = time.perf_counter()
    boxes = ci.batch_boxes(args.batch_boxes, seed=3)
    ps, off = pl.concat(boxes)
    gen_s = time.perf_counter() - t0
    ctx = Context(0)
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, prec, kappa_max=args.kappa)
    io = ctx.step_buffers(dev)
    npairs, _ = ctx.step(io, prm, box_offsets=off)
    ppp = npairs / ps.n
    if args.autotune_batch:
        tuned, tune_ms = at.tune(ctx, dev, prm, with_hsolve=False, box_offsets=off,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
        if args.tune_out:
            at.save(prec, ppp, tuned, tune_ms, f"{args.batch_boxes} boxes, sides 8..48",
                    args.tune_out, kind="batch")
    else:
        tuned = at.load(prec, ppp, kind="batch")
        if tuned:
            at.apply(ctx, tuned)
    # eager steps (per-kernel event times), then the recorded step
    for _ in range(args.warmup):
        ctx.step(io, prm, box_offsets=off)
    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        ctx.step(io, prm, box_offsets=off)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t1) * 1e3 / max(args.steps, 1)
    kern = {}
    for k in ("sort", "k_walk", "k_compact_rows", "k_walk_long", "k_extra_rank", "k_volume",
              "k_moments", "k_corrections", "k_gradv", "k_deriv", "k_deriv_fix"):
        ms, cnt = ctx.timing_read(k)
        kern[k] = ms / max(cnt, 1)
    ctx.timing(False)
    g_ms, st, info = graph_replay_ms(ctx, io, prm, args.steps, args.warmup, box_offsets=off)
    ctx.graph_destroy()
    out = {"workload": f"{args.batch_boxes} periodic boxes, side n_b = round(exp U(ln 8, ln 48)), "
                       f"half jittered lattice, half lognormal (sigma 1.5, P(k)~k^-2, H <= 0.3 L), "
                       f"gamma-law gas rho, u log-uniform in [0.1, 10], seed 3; {precision_name}",
           "boxes": args.batch_boxes, "particles": ps.n, "pairs_per_step": int(info["n_pairs"]),
           "graph_ms_per_step": g_ms, "graph_pairs_per_s": info["n_pairs"] / (g_ms * 1e-3),
           "eager_ms_per_step": eager_ms, "graph_status": st, "graph_info": info,
           "lanes": tuned, "kernel_ms": kern, "generate_seconds": gen_s}
    if not args.no_check:
        ref = ctx.step_buffers(dev)
        ctx.step(ref, pl.params_for(ps, 64.0, CRK_FP64), box_offsets=off)
        torch.cuda.synchronize()
        errs = {}
        for k in OUT_KEYS:
            a, b = io[k], ref[k]
            den = b.abs().max().item()
            errs[k] = (a - b).abs().max().item() / den if den > 0 else (a - b).abs().max().item()
        out["max_rel_err_vs_fp64"] = errs
        out["err_target_met"] = bool(max(errs.values()) <= 1e-5)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-side", type=int, default=128)
    ap.add_argument("--precision", choices=("mixed", "adapt", "fp64"), default="adapt")
    ap.add_argument("--cpu-n-side", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-hsurrogate", action="store_true",
                    help="skip the smoothing-length network leg (train + plain vs seeded iteration)")
    ap.add_argument("--hs-train-sides", type=str, default="64,80,96,112,128",
                    help="sides of the network's training boxes (each labelled cold and warm)")
    ap.add_argument("--hs-eval-side", type=int, default=128)
    ap.add_argument("--hs-steps", type=int, default=1500)
    ap.add_argument("--lanes", type=str, default="", help="vol,mom,grad,der lanes per particle")
    ap.add_argument("--walk", type=str, default="", help="lanes,cap of the neighbour walk")
    ap.add_argument("--autotune", action="store_true",
                    help="tune lanes per pass on this workload before timing")
    ap.add_argument("--tune-out", type=str, default="",
                    help="write the tuned table to this path (with --autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device-to-device copy three times (scales HBM counters)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the HIP-graph replay timing of the step")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-box batch leg")
    ap.add_argument("--no-full-size", action="store_true", help="skip the 256^3 full-step leg")
    ap.add_argument("--no-timestep", action="store_true",
                    help="skip the leg timing the Courant terms fused into the derivative pass")
    ap.add_argument("--no-compat", action="store_true",
                    help="skip the leg timing the compatible energy pass")
    ap.add_argument("--no-verlet", action="store_true",
                    help="skip the leg timing velocity-Verlet hydro steps")
    ap.add_argument("--no-nres268", action="store_true",
                    help="skip the sensitivity point at N_res = 268")
    ap.add_argument("--no-leaves", action="store_true",
                    help="skip the RCB leaf-tiling comparison")
    ap.add_argument("--full-side", type=int, default=256)
    ap.add_argument("--batch-boxes", type=int, default=512)
    ap.add_argument("--autotune-batch", action="store_true",
                    help="tune the lanes on the batch workload (stored with --tune-out)")
    ap.add_argument("--kappa", type=float, default=1000.0,
                    help="conditioning bound above which the adaptive mode runs a row in FP64")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the CRKSPH passes here run on a single MI355X; "
              "multi-GPU sharding is a design note only. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_launch": (1 << 28) * 8}), flush=True)
        return
    from paper_2202_02840_amd import CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT, Context
    from paper_2202_02840_amd import pipeline as pl

    ps = make_workload(args.n_side)
    prec = {"mixed": CRK_MIXED, "adapt": CRK_MIXED_ADAPT, "fp64": CRK_FP64}[args.precision]
    ctx = Context(0)
    if args.lanes:
        ctx.set_lanes(*[int(v) for v in args.lanes.split(",")])
    if args.walk:
        ctx.set_walk(*[int(v) for v in args.walk.split(",")])
    dev = pl.upload(ps)
    prm = pl.params_for(ps, 64.0, prec, kappa_max=args.kappa)
    torch.cuda.synchronize()

    # lanes per pass: tuned now, or from the stored table for this workload class
    from paper_2202_02840_amd import autotune as at
    first = pl.step(ctx, dev, prm, count_singular=False)
    ppp = first["n_pairs"] / ps.n
    tuned = None
    if args.autotune:
        tuned, tune_ms = at.tune(ctx, dev, prm, log=lambda s: print(s, file=sys.stderr, flush=True))
        if args.tune_out:
            at.save(prec, ppp, tuned, tune_ms, f"lognormal {args.n_side}^3 sigma 1.5", args.tune_out)
    elif not (args.lanes or args.walk):
        tuned = at.load(prec, ppp)
        if tuned:
            at.apply(ctx, tuned)

    for _ in range(args.warmup):
        out = pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    # HIP events bracket only the derivative pass inside the timed region
    # (its time is the roofline's); the per-kernel breakdown comes from
    # further steps after it, where every kernel is bracketed
    ctx.timing(True)
    ctx.timing_only("k_deriv")
    ctx.timing_reset()
    torch.cuda.synchronize()
    # every step is timed on its own (synchronised); the line reports the
    # median step, and the mean over the whole timed region beside it
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        out = pl.step(ctx, dev, prm, count_singular=False)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
    t1 = time.perf_counter()
    ms_mean = (t1 - t0) * 1e3 / max(args.steps, 1)
    ms_step = float(np.median(step_ms))
    ms, cnt = ctx.timing_read("k_deriv")
    deriv_ms = ms / max(cnt, 1)
    ctx.timing_only(None)
    ctx.timing_reset()
    for _ in range(BREAKDOWN_STEPS):
        out = pl.step(ctx, dev, prm, count_singular=False)
    torch.cuda.synchronize()
    kern = {}
    for k in ("sort", "k_walk", "k_compact_rows", "k_walk_long", "k_extra_rank", "k_volume", "k_moments",
              "k_corrections", "k_flag", "k_pack", "k_gradv", "k_gradv_fix", "k_deriv",
              "k_deriv_fix"):
        ms, cnt = ctx.timing_read(k)
        kern[k] = ms / max(cnt, 1)
    ctx.timing(False)
    fp64_rows = ctx.adaptive_rows() if prec == CRK_MIXED_ADAPT else (0, 0)
    npairs = int(out["n_pairs"])
    n = ps.n

    # roofline of the dominant kernel (the derivative pass), timed in the
    # timed region
    t_der = deriv_ms * 1e-3
    flops = DERIV_FLOPS_PER_PAIR * npairs
    key = "fp64" if prec == CRK_FP64 else "mixed"
    bytes_alg = DERIV_BYTES_PER_PARTICLE[key] * n + DERIV_BYTES_PER_PAIR * npairs
    achieved_tf = flops / t_der / 1e12
    hbm_gbs = bytes_alg / t_der / 1e9

    # the same step recorded as one HIP graph and replayed
    graph = None
    if not args.no_graph:
        io = ctx.step_buffers(dev)
        g_ms, g_st, g_info = graph_replay_ms(ctx, io, prm, args.steps, args.warmup)
        ctx.graph_destroy()
        same = all(torch.equal(io[k], out[k]) for k in OUT_KEYS)
        graph = {"ms_per_step": g_ms, "pairs_per_s": g_info["n_pairs"] / (g_ms * 1e-3),
                 "status": g_st, "n_pairs": g_info["n_pairs"], "bitwise_equal_to_eager": same}
        del io

    # accuracy of this path against the FP64 GPU path at full size
    errs = errs_comp = errs_elem = None
    if not args.no_check:
        ref = pl.step(ctx, dev, pl.params_for(ps, 64.0, CRK_FP64), count_singular=False)
        cur = pl.step(ctx, dev, prm, count_singular=False)
        torch.cuda.synchronize()
        errs, errs_comp, errs_elem = {}, {}, {}
        for k in OUT_KEYS:
            a, b = cur[k], ref[k]
            den = b.abs().max().item()
            errs[k] = (a - b).abs().max().item() / den if den > 0 else (a - b).abs().max().item()
            # each component on its own scale, and element by element where
            # |ref| exceeds 1e-6 of the output's largest value
            a2, b2 = a.reshape(-1, a.shape[-1]), b.reshape(-1, b.shape[-1])
            worst = 0.0
            for c in range(b2.shape[0]):
                dc = b2[c].abs().max().item()
                e = (a2[c] - b2[c]).abs().max().item()
                worst = max(worst, e / dc if dc > 0 else e)
            errs_comp[k] = worst
            big = b.abs() > 1e-6 * den
            errs_elem[k] = ((a - b).abs()[big] / b.abs()[big]).max().item() if bool(big.any()) else 0.0

    line = {
        "metric": "CRKSPH pair-interactions/s at <=1e-5 rel err vs FP64; % HBM roofline",
        "value": npairs / (ms_step * 1e-3),
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_mean": ms_mean,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == CRK_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"lognormal clustered gas, {args.n_side}^3 = {n} particles, "
                               f"sigma_ln_rho 1.5, P(k)~k^-2, 64-neighbour H, seed 2; "
                               f"{args.precision} CRKSPH step",
                   "particles": n, "pairs_per_step": npairs,
                   "mean_pairs_per_particle": npairs / n, "precision": args.precision,
                   "kappa_max": args.kappa if prec == CRK_MIXED_ADAPT else None,
                   "fp64_rows": fp64_rows[0], "fp64_touched_rows": fp64_rows[1],
                   "lanes": tuned},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / VALU_PEAK_TFLOPS,
                     "traffic": deriv_traffic(args.precision, (tuned or {}).get("der_wave", 8)),
                     "traffic_unit": "bytes per launch", "algorithmic_bytes": bytes_alg,
                     "kernel": "k_deriv", "kernel_ms": deriv_ms,
                     "flops_per_pair": DERIV_FLOPS_PER_PAIR,
                     "frac_of_packed_fp32_peak": achieved_tf / VALU_PEAK_PACKED_FP32,
                     "hbm_algorithmic_gbs": hbm_gbs, "hbm_frac": hbm_gbs / HBM_PEAK_GBS},
        "kernel_ms": kern,
        "kernel_ms_steps": BREAKDOWN_STEPS,
        "workspace_bytes": ctx.workspace_bytes(),
        "max_rel_err_vs_fp64": errs,
        "max_rel_err_vs_fp64_per_component": errs_comp,
        "max_elementwise_rel_err_vs_fp64": errs_elem,
        "elementwise_floor": "elements with |ref| > 1e-6 max |ref| of the output",
        "err_target_met": None if errs is None else bool(max(errs.values()) <= 1e-5),
        "graph_replay": graph,
    }
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    log(f"main step {ms_step:.3f} ms")
    if not args.no_timestep:
        line["timestep"] = timestep_leg(ctx, dev, prm, args)
        log(f"timestep leg: derivative pass {line['timestep']['k_deriv_ms']:.3f} ms with the terms")
    if not args.no_compat:
        line["compatible_energy"] = compat_leg(ctx, dev, prm, args, deriv_ms)
        log(f"compatible energy leg: {line['compatible_energy']['k_compat_ms']:.3f} ms")
    if not args.no_verlet:
        line["verlet"] = verlet_leg(ctx, args, prec)
        log(f"verlet leg: {line['verlet']['eng']['ms_per_step']:.3f} ms per step "
            f"({line['verlet']['compat']['ms_per_step']:.3f} with the compatible energy)")
    if not args.no_nres268:
        line["nres268"] = nres268_leg(args, prec)
        log(f"N_res = 268 leg: {line['nres268']['ms_per_step']:.3f} ms per step, "
            f"{line['nres268']['mean_pairs_per_particle']:.0f} pairs per particle")
    if not args.no_leaves:
        line["rcb_leaves"] = {"c2": leaves_leg(args, prec, args.n_side, 1.5, -2.0, 2, False,
                                               f"lognormal {args.n_side}^3, sigma 1.5, P(k)~k^-2, seed 2")}
        log(f"leaves leg: build {line['rcb_leaves']['c2']['rcb']['build_ms_median_of_3']:.3f} ms "
            f"(Morton {line['rcb_leaves']['c2']['morton']['build_ms_median_of_3']:.3f} ms)")
        if not args.no_full_size:
            line["rcb_leaves"]["c5"] = leaves_leg(
                args, prec, args.full_side, 2.0, -2.5, 5, True,
                f"lognormal {args.full_side}^3 sigma 2.0, P(k)~k^-2.5, 1% in 64 clumps, seed 5; "
                "the generator's supports")
            log(f"leaves leg (clumps): build {line['rcb_leaves']['c5']['rcb']['build_ms_median_of_3']:.3f} ms "
                f"(Morton {line['rcb_leaves']['c5']['morton']['build_ms_median_of_3']:.3f} ms)")
    if not args.no_batch:
        line["batch"] = batch_leg(args, prec, args.precision)
        log(f"batch leg {line['batch']['graph_ms_per_step']:.3f} ms per replay")
    theta = None
    if not args.no_hsurrogate:
        line["h_surrogate"], theta = hsurrogate_leg(ctx, args)
        log(f"h-surrogate leg speedup {line['h_surrogate']['speedup']:.3f}")
    if not args.no_full_size:
        del ctx, dev, out
        torch.cuda.empty_cache()
        line["full_size"] = full_size_leg(args, prec, theta)
        log(f"full-size leg step {line['full_size']['step_ms']:.3f} ms")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_n_side)
        log("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
