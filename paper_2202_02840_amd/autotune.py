"""Autotuner for the lanes-per-particle of every pass (and the particles
per wavefront of the derivative pass's balanced mapping).

Each pair pass, the neighbour walk and the smoothing-length iteration split a
particle's work over a group of G lanes of a wave64 (crk_set_lanes,
crk_set_walk, crk_set_hsolve); the walk also picks how coarse a cell level
it walks (fewer cells against more candidates). The best G depends on the neighbour counts
and on the precision, so the tuner times every candidate on the actual
workload with the library's own per-kernel HIP-event timers, one knob at a
time (coordinate descent from the current setting), and keeps the fastest.
Results are stored in a JSON table keyed by precision and mean pairs per
particle, which bench.py and callers apply with :func:`apply`.
"""
from __future__ import annotations

import json
import os

import torch

from ._lib import Context
from . import pipeline as pl

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tune_table.json")

DEFAULT = {"walk": 8, "walk_level": 0, "vol": 4, "mom": 1, "grad": 4, "der": 8, "vol_wave": 0,
           "mom_wave": 0, "grad_wave": 0, "der_wave": 8, "hsolve": 16}
CANDIDATES = {
    "walk": (2, 4, 8, 16),
    "walk_level": (0, 1, 2),
    "vol": (1, 2, 4, 8, 16),
    "mom": (1, 2, 4, 8),
    "grad": (2, 4, 8, 16),
    "der": (4, 8, 16, 32),
    "vol_wave": (0, 4, 8, 16),
    "mom_wave": (0, 4, 8, 16),
    "grad_wave": (0, 4, 8, 16),
    "der_wave": (0, 4, 8, 16),
    "hsolve": (4, 8, 16, 32),
}
KERNEL = {"walk": "k_walk", "walk_level": "k_walk", "vol": "k_volume", "mom": "k_moments", "grad": "k_gradv",
          "der": "k_deriv", "vol_wave": "k_volume", "mom_wave": "k_moments", "grad_wave": "k_gradv",
          "der_wave": "k_deriv"}


def key_for(precision: int, pairs_per_particle: float, kind: str = "") -> str:
    """Table key: precision, mean pairs per particle rounded to 16, and the
    workload kind ("" for one box, "batch" for many small boxes)."""
    k = f"p{precision}/n{int(round(pairs_per_particle / 16.0)) * 16}"
    return f"{k}/{kind}" if kind else k


def _kind(key: str) -> str:
    parts = key.split("/")
    return parts[2] if len(parts) > 2 else ""


def apply(ctx: Context, cfg: dict) -> None:
    ctx.set_lanes(cfg["vol"], cfg["mom"], cfg["grad"], cfg["der"])
    # volume, moment, velocity-gradient and derivative passes: balanced lane
    # groups of *_wave particles per wave (0: the lanes per particle above);
    # tables written before the knobs existed take the defaults
    ctx.set_wave_mapping(*(cfg.get(k, DEFAULT[k]) for k in ("vol_wave", "mom_wave", "grad_wave",
                                                             "der_wave")))
    ctx.set_walk(cfg["walk"], 0, cfg.get("walk_level", 0))
    ctx.set_hsolve(cfg["hsolve"], 0, 0, 0.0)


def load(precision: int, pairs_per_particle: float, kind: str = "") -> dict | None:
    if not os.path.exists(TABLE):
        return None
    tab = json.load(open(TABLE))
    k = key_for(precision, pairs_per_particle, kind)
    if k in tab:
        return dict(tab[k]["config"])
    # nearest neighbour-count class of the same precision (and kind, if any)
    same = [kk for kk in tab if kk.startswith(f"p{precision}/")]
    if any(_kind(kk) == kind for kk in same):
        same = [kk for kk in same if _kind(kk) == kind]
    if not same:
        return None
    best = min(same, key=lambda kk: abs(int(kk.split("/")[1][1:]) - pairs_per_particle))
    return dict(tab[best]["config"])


def _time_step(ctx, dev, prm, kernel: str, reps: int, box_offsets=None) -> float:
    pl.step(ctx, dev, prm, count_singular=False, box_offsets=box_offsets)   # settle allocations
    ctx.timing(True)
    ctx.timing_reset()
    for _ in range(reps):
        pl.step(ctx, dev, prm, count_singular=False, box_offsets=box_offsets)
    torch.cuda.synchronize()
    ms, cnt = ctx.timing_read(kernel)
    ctx.timing(False)
    return ms / max(cnt, 1)


def _time_hsolve(ctx, dev, prm, nres: float, reps: int) -> float:
    ctx.build_cells(dev["x"], dev["y"], dev["z"], dev["H"], prm)
    Hs = ctx.permute(dev["H"], True)
    best = None
    for _ in range(reps):
        ctx.timing(True)
        ctx.timing_reset()
        ctx.hsolve(nres, Hs, 1e-8, 1000)
        torch.cuda.synchronize()
        ms, _ = ctx.timing_read("k_hsolve")
        ctx.timing(False)
        ctx.update_support(Hs)
        best = ms if best is None else min(best, ms)
    return best


def tune(ctx: Context, dev: dict, prm, nres: float = 64.0, start: dict | None = None,
         reps: int = 3, with_hsolve: bool = True, log=print, box_offsets=None) -> tuple[dict, dict]:
    """Coordinate descent over the knobs; returns (best config, timings)."""
    cfg = dict(start or DEFAULT)
    timings = {}
    for knob, cands in CANDIDATES.items():
        if knob == "hsolve" and not with_hsolve:
            continue
        res = {}
        for g in cands:
            trial = dict(cfg)
            trial[knob] = g
            apply(ctx, trial)
            if knob == "hsolve":
                res[g] = _time_hsolve(ctx, dev, prm, nres, max(1, reps - 1))
            else:
                res[g] = _time_step(ctx, dev, prm, KERNEL[knob], reps, box_offsets)
        best = min(res, key=res.get)
        cfg[knob] = best
        timings[knob] = {str(k): v for k, v in res.items()}
        if log:
            log(f"tune {knob}: {res} -> {best}")
    apply(ctx, cfg)
    return cfg, timings


def save(precision: int, pairs_per_particle: float, cfg: dict, timings: dict, workload: str,
         path: str = TABLE, kind: str = "") -> None:
    tab = json.load(open(path)) if os.path.exists(path) else {}
    tab[key_for(precision, pairs_per_particle, kind)] = {"config": cfg, "timings_ms": timings,
                                                         "workload": workload}
    with open(path, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
