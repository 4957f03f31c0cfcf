"""Time integration with the velocity-Verlet hydro operator (eq. verletOP).

Each step re-solves the support radii for the current positions (eqs. hi,
thacker: one cell build and the h iteration), then advances the state with
crk_verlet_step: half kick and drift with the derivatives carried over from
the previous step's end evaluation, one whole evaluation at the predicted
state, closing half kick. The first step evaluates its start derivatives.
Every array stays on the device in the caller's order.
"""
from __future__ import annotations

import math

import torch

from ._lib import Context, Params


def update_support(ctx: Context, state: dict, params: Params, nres: float, tol: float = 1e-6,
                   max_iter: int = 200) -> int:
    """H of every particle re-solved for the current positions (in place);
    returns the number not converged."""
    ctx.build_cells(state["x"], state["y"], state["z"], state["H"], params)
    Hs = ctx.permute(state["H"], True)
    Hn, _, nun = ctx.hsolve(nres, Hs, tol, max_iter)
    state["H"].copy_(ctx.permute(Hn, False))
    return nun


def evolve(ctx: Context, state: dict, params: Params, t_end: float, dt: float,
           nres: float = 64.0, h_tol: float = 1e-6, log=None, energy: str = "eng") -> dict:
    """Fixed steps of at most dt from t = 0 to t_end. state holds x, y, z, H,
    v, m, u (optional rho); dpdt and dudt are added. energy: "eng" (du/dt of
    eq. eng) or "compat" (the compatible update per half kick). Returns a
    summary."""
    n = state["x"].shape[0]
    state.setdefault("dpdt", torch.zeros(3, n, dtype=torch.float64, device=state["x"].device))
    state.setdefault("dudt", torch.zeros(n, dtype=torch.float64, device=state["x"].device))
    nsteps = max(1, int(math.ceil(t_end / dt - 1e-9)))
    h = t_end / nsteps
    unconverged = 0
    for k in range(nsteps):
        unconverged += update_support(ctx, state, params, nres, h_tol)
        ctx.verlet_step(state, params, h, start_eval=(k == 0), energy=energy)
        if log and (k + 1) % max(1, nsteps // 5) == 0:
            log(f"step {k + 1}/{nsteps}")
    return {"steps": nsteps, "dt": h, "h_unconverged": unconverged}
