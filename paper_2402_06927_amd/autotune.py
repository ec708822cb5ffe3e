"""Tile autotuner of the model kernels.

A particle's row of nx nodes is split over NT threads (a power of two,
64..512) holding nx / NT nodes each (4, 8 or 16 register slots; 2 on one
wavefront for nx <= 128).  For a grid
size the tuner times the library's ensemble step (``sch_ensemble_step``, the
kernel every filter stage reruns) on the caller's own ensemble for every
tile the library provides, keeps the fastest, and can cache the choice per
grid size in a JSON file.  The choice is applied through the library's
SCH_TUNE_THREADS knob.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import sch

# (threads per particle, register slots) of the compiled model kernels
TILES = ((64, 2), (64, 4), (64, 8), (64, 16), (128, 8), (128, 16), (256, 8), (256, 16), (512, 8),
         (512, 16))


def slots(nx: int, nt: int) -> int:
    need = math.ceil(nx / nt)
    if nt == 64 and need <= 2:
        return 2
    return 4 if need <= 4 else (8 if need <= 8 else 16)


def candidates(nx: int) -> list[int]:
    """Thread counts with a compiled kernel for this grid size."""
    out = []
    for nt in (64, 128, 256, 512):
        if nx < nt or math.ceil(nx / nt) > 16:
            continue
        if (nt, slots(nx, nt)) in TILES:
            out.append(nt)
    return out


def load_cache(path: str | None) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return {int(k): int(v) for k, v in json.load(f).items()}


def save_cache(path: str, table: dict):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({str(k): v for k, v in sorted(table.items())}, f, indent=1)
    os.replace(tmp, path)


def tune(model: sch.Model, m: torch.Tensor, u: torch.Tensor, n_steps: int = 6, reps: int = 3,
         cache: str | None = None, apply: bool = True) -> tuple[int, dict]:
    """Fastest thread count for the grid of `model` on the ensemble (m, u)
    (not modified: copies are stepped; per tile the best of `reps` timed
    windows of n_steps steps).  Returns (threads, {threads: ms})."""
    nx = model.nx
    table = load_cache(cache)
    if nx in table and table[nx] in candidates(nx):
        best = table[nx]
        if apply:
            sch.sch_tune_set(sch.TUNE_THREADS, best)
        return best, {}
    n = m.shape[0]
    dW = torch.zeros((n, n_steps, model.n_modes), dtype=torch.float64, device=m.device)
    timing = {}
    for nt in candidates(nx):
        sch.sch_tune_set(sch.TUNE_THREADS, nt)
        mm, uu = m.clone(), u.clone()
        sch.sch_ensemble_step(model, mm, uu, dW)  # warm-up
        best_ms = float("inf")
        for _ in range(reps):
            mm.copy_(m)
            uu.copy_(u)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sch.sch_ensemble_step(model, mm, uu, dW)
            e1.record()
            torch.cuda.synchronize()
            best_ms = min(best_ms, e0.elapsed_time(e1))
        timing[nt] = best_ms
    best = min(timing, key=timing.get)
    sch.sch_tune_set(sch.TUNE_THREADS, best if apply else 0)
    if cache:
        table[nx] = best
        save_cache(cache, table)
    return best, timing


def tile_key(nx: int) -> tuple:
    """Instances whose grids share this key have the same compiled tiles to
    choose from."""
    return tuple((nt, slots(nx, nt)) for nt in candidates(nx))


def tune_batch(make_model, nxs, n_particles: int = 1024, cache: str | None = None,
               seed: int = 1) -> dict[int, int]:
    """Threads per particle for every grid size in `nxs` (the instances of a
    batch): grids are grouped by their tile options, each group is tuned once
    at its median grid on a sample ensemble of `n_particles` (smooth random
    states; enough workgroups to fill the chip for every tile, so that the
    smaller tiles are not timed on a half-empty GPU), and the choice
    applies to the whole group.  `make_model(nx)`
    returns an sch.Model for grid nx.  Leaves SCH_TUNE_THREADS unset."""
    import numpy as np

    groups: dict[tuple, list[int]] = {}
    for nx in sorted(set(int(x) for x in nxs)):
        groups.setdefault(tile_key(nx), []).append(nx)
    choice = {}
    g = np.random.default_rng(seed)
    for key, members in groups.items():
        if len(key) == 1:
            best = key[0][0]
        else:
            nx = members[len(members) // 2]
            model = make_model(nx)
            x = np.arange(nx) / nx
            u = np.stack([0.2 / np.cosh((x - 0.5) * 20.0 + 0.1 * g.standard_normal()) ** 2
                          for _ in range(n_particles)])
            ut = torch.tensor(u, dtype=torch.float64, device="cuda")
            mt = torch.empty_like(ut)
            sch.sch_init_momentum(model, ut, mt)
            best, _ = tune(model, mt, ut, cache=cache, apply=False)
        for nx in members:
            choice[nx] = best
    return choice
