"""Sequencing of the C-ABI calls for one CRKSPH step (no arithmetic here).

One step is: crk_build_cells -> crk_moments -> crk_corrections ->
crk_derivatives, which covers the cell/neighbour build, volumes, moments, RK
corrections, velocity gradient and the momentum/energy derivatives.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import CRK_FP64, CRK_MIXED, Context, Params


def upload(ps, device="cuda") -> dict:
    """Particle set (numpy, original order) -> float64 device tensors."""
    t = lambda a: None if a is None else torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
    return dict(x=t(ps.x), y=t(ps.y), z=t(ps.z), H=t(ps.H), m=t(ps.m), u=t(ps.u), v=t(ps.v),
                rho=t(ps.rho))


def params_for(ps, nres: float = 64.0, precision: int = CRK_FP64, **over) -> Params:
    p = Params.default(nres, L=ps.L, gamma=ps.gamma, precision=precision)
    for k, v in over.items():
        setattr(p, k, v)
    return p


def concat(boxes) -> tuple:
    """Particle sets of a batch -> one concatenated set and the box offsets."""
    import crk_inputs as ci
    off = np.concatenate([[0], np.cumsum([b.n for b in boxes])]).astype(np.int64)
    cat = lambda k: np.concatenate([getattr(b, k) for b in boxes])
    rho = None if any(b.rho is None for b in boxes) else cat("rho")
    ps = ci.ParticleSet(cat("x"), cat("y"), cat("z"), cat("H"), cat("m"), cat("u"),
                        np.concatenate([b.v for b in boxes], axis=1), rho, L=boxes[0].L,
                        gamma=boxes[0].gamma, meta=dict(kind="batch", boxes=len(boxes)))
    return ps, off


def step(ctx: Context, dev: dict, params: Params, cell_size: float = 0.0,
         count_singular: bool = True, box_offsets=None, timestep: bool = False,
         compat_dt: float = None) -> dict:
    """All passes of one step; every returned array is in cell-sorted order.
    With box_offsets (host, nboxes+1) the arrays hold a batch of boxes. With
    timestep the Courant terms (vsig, csq, vmax, dt_hyd) come along; with
    compat_dt the compatible energy update over that step (du_compat)."""
    if box_offsets is None:
        perm, npairs = ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], params, cell_size)
    else:
        perm, npairs = ctx.build_cells_batch(box_offsets, dev["x"], dev["y"], dev["z"], dev["H"],
                                             params, cell_size)
    mom = ctx.moments(params)
    corr = ctx.corrections(mom, count_singular=count_singular)
    v = ctx.permute(dev["v"], True)
    m = ctx.permute(dev["m"], True)
    u = ctx.permute(dev["u"], True)
    rho = None if dev.get("rho") is None else ctx.permute(dev["rho"], True)
    if timestep:
        ctx.set_timestep(True)
    der = ctx.derivatives(params, v, m, u, rho, mom["V"], corr)
    out = dict(perm=perm, n_pairs=npairs)
    out.update(mom)
    out.update(corr)
    out.update(der)
    if timestep:
        out.update(ctx.timestep(params, u, m, rho, mom["V"], der["gradv"]))
        ctx.set_timestep(False)
    if compat_dt is not None:
        out["du_compat"] = ctx.compatible_energy(params, v, m, u, rho, mom["V"], corr, der["gradv"],
                                                 der["dpdt"], compat_dt)
    return out


def to_original(out: dict, perm: torch.Tensor) -> dict:
    """Sorted-order device results -> numpy arrays in the original order."""
    p = perm.long().cpu().numpy()
    res = {}
    for k, v in out.items():
        if isinstance(v, torch.Tensor) and k != "perm":
            a = v.cpu().numpy()
            b = np.empty_like(a)
            b[..., p] = a
            res[k] = b
        else:
            res[k] = v
    return res


__all__ = ["upload", "params_for", "step", "to_original", "concat", "CRK_FP64", "CRK_MIXED"]
