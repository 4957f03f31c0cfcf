"""Training and use of the smoothing-length network (sequencing of C-ABI
calls only: features, targets, gradients, Adam and the iteration itself all
run in libcrk.so).

Training pairs come from the plain iteration of eq. (thacker): for a box
with starting support radii H_prev, the features at H_prev and the target
ln(H_conv / H_prev), H_conv being the converged radius. At use, the network
proposes H_seed = H_prev exp(y) and the same plain iteration finishes from
there; the iteration alone decides the converged H.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from ._lib import CRK_FP64, Context
from . import pipeline as pl


def training_pairs(ctx: Context, ps, nres: float = 64.0, tol: float = 1e-7, max_iter: int = 1000):
    """(features [8, n] float, targets [n] float, iterations [n]) for one box."""
    dev = pl.upload(ps)
    ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], pl.params_for(ps, nres, CRK_FP64))
    Hs = ctx.permute(dev["H"], True)
    feat = ctx.hnet_features(nres, Hs)
    Hc, it, nun = ctx.hsolve(nres, Hs, tol, max_iter)
    tgt = ctx.hnet_targets(Hs, Hc)
    return feat, tgt, it


def moved(ps, H_conv: np.ndarray, courant: float = 0.25, nres: float = 64.0):
    """The box one Courant step later: every particle moved by v dt with
    dt = courant * median(H / n_h) / max |v| (wrapped into the box), its
    starting support the converged H before the move (a warm start)."""
    import crk_inputs as ci
    nh = (3.0 * nres / (4.0 * np.pi)) ** (1.0 / 3.0)
    vmax = float(np.sqrt((ps.v ** 2).sum(axis=0)).max())
    dt = courant * float(np.median(H_conv / nh)) / max(vmax, 1e-30)
    wrap = lambda a: np.mod(a, ps.L)
    q = ci.ParticleSet(wrap(ps.x + ps.v[0] * dt), wrap(ps.y + ps.v[1] * dt), wrap(ps.z + ps.v[2] * dt),
                       np.asarray(H_conv, dtype=np.float64).copy(), ps.m, ps.u, ps.v, ps.rho, L=ps.L,
                       gamma=ps.gamma, meta=dict(ps.meta, moved_dt=dt))
    # a coordinate that rounds to L after the wrap goes to 0
    for a in (q.x, q.y, q.z):
        a[a >= ps.L] = 0.0
    return q


def converged(ctx: Context, ps, nres: float = 64.0, tol: float = 1e-7, max_iter: int = 1000):
    """Converged supports of a box in its original order (plain iteration
    from the box's own H)."""
    dev = pl.upload(ps)
    perm, _ = ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], pl.params_for(ps, nres, CRK_FP64))
    Hs = ctx.permute(dev["H"], True)
    Hc, it, nun = ctx.hsolve(nres, Hs, tol, max_iter)
    Ho = torch.empty_like(Hc)
    Ho[perm.long()] = Hc
    return Ho.cpu().numpy()


def train(ctx: Context, theta0: np.ndarray, feats, targets, steps: int = 2000, batch: int = 4096,
          lr: float = 3e-3, lr_end: float = 1e-4, seed: int = 0, log_every: int = 0):
    """Adam on mean squared error over the concatenated pairs; batches are
    drawn by a seeded permutation. Returns (theta tensor, loss history)."""
    F = torch.cat(feats, dim=1).contiguous()
    T = torch.cat(targets).contiguous()
    N = T.shape[0]
    theta = torch.as_tensor(np.asarray(theta0, dtype=np.float32), device=ctx.device).contiguous()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    g = np.random.default_rng(seed)
    hist = []
    order = torch.as_tensor(g.permutation(N), device=ctx.device)
    pos = 0
    for step in range(1, steps + 1):
        if pos + batch > N:
            order = torch.as_tensor(g.permutation(N), device=ctx.device)
            pos = 0
        idx = order[pos:pos + batch]
        pos += batch
        fb = F.index_select(1, idx).contiguous()
        tb = T.index_select(0, idx).contiguous()
        frac = (step - 1) / max(steps - 1, 1)
        lr_s = lr * (lr_end / lr) ** frac                 # geometric decay
        want = bool(log_every) and step % log_every == 0
        _, loss = ctx.hnet_train_step(theta, m, v, step, lr_s, fb, tb, want_loss=want)
        if want:
            hist.append((step, loss))
    return theta, hist


def evaluate(ctx: Context, ps, theta, nres: float = 64.0, tol: float = 1e-7, max_iter: int = 1000,
             repeats: int = 1) -> dict:
    """Plain iteration from H_prev against network seed + iteration, on the
    same box: iterations, wall time of each (GPU, synchronised) and the
    largest relative difference of the converged H."""
    dev = pl.upload(ps)
    prm = pl.params_for(ps, nres, CRK_FP64)
    ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], prm)
    Hs = ctx.permute(dev["H"], True)
    out = {}
    for name in ("plain", "surrogate"):
        best = None
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            start = Hs if name == "plain" else ctx.hnet_seed(theta, nres, Hs)
            Hc, it, nun = ctx.hsolve(nres, start, tol, max_iter)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, Hc, it, nun)
            # hsolve moved the context's supports: restore the start state
            ctx.update_support(Hs)
        dt, Hc, it, nun = best
        itn = it.double()
        out[name] = dict(seconds=dt, mean_iters=float(itn.mean()), max_iters=int(it.max()),
                         p99_iters=float(torch.quantile(itn, 0.99).item()),
                         p999_iters=float(torch.quantile(itn, 0.999).item()),
                         unconverged=int(nun), H=Hc)
    out["max_rel_dH"] = float(((out["surrogate"]["H"] / out["plain"]["H"]) - 1).abs().max())
    out["speedup"] = out["plain"]["seconds"] / out["surrogate"]["seconds"]
    for k in ("plain", "surrogate"):
        out[k].pop("H")
    return out
