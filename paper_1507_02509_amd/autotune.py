"""Tile-shape autotuner for the step and ensemble kernels.

For a single lattice it times every candidate launch configuration -- the
single-step kernel with each tile (width, rows per thread, non-temporal
stores) and the two-step fused kernel with each tile height and store kind --
on the caller's own lattice with HIP events; for an ensemble, every tile of
the ensemble kernel.  It keeps the one with the smallest median time and
caches the choice in a JSON file keyed by the device name and the
configuration (form, collision, variant, stabiliser mode and guard, lattice
sizes).
The lattice state is restored afterwards: every trial takes an even number of
steps and the state buffers are copied back, so tuning changes nothing but
the tile.  Results of the step kernels are bitwise identical for every tile,
so the choice only affects speed.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import _lib

STEP_TILES = [(w, r, nt) for (w, r) in ((64, 1), (64, 4), (128, 1), (128, 2), (128, 4), (256, 1), (256, 2))
              for nt in (False, True)]
ENSEMBLE_TILES = [(w, r, nt) for (w, r) in ((128, 2), (256, 1), (256, 2)) for nt in (False, True)]
ENSEMBLE_CANDIDATES = ([("single",) + t for t in ENSEMBLE_TILES] +
                       [("fused", rows, nt) for rows in (8, 16) for nt in (False, True)])
# launch configurations of a single lattice: ("single", width, rows per
# thread, nt) or ("fused", tile rows, nt) (two steps per launch)
STEP_CANDIDATES = ([("single",) + t for t in STEP_TILES] +
                   [("fused", rows, nt) for rows in (8, 16, 24, 32) for nt in (False, True)])


def apply_config(sim, cand):
    """Set a launch configuration from STEP_CANDIDATES on a Sim."""
    if cand[0] == "single":
        sim.set_fusion(1)
        sim.set_tile(*cand[1:])
    else:
        sim.set_fusion(2, cand[1])   # raises for a 32-row FP64 tile (skipped by the tuner)
        sim.set_tile(256, 1, cand[2])   # the tile of an odd remaining single step


def cache_path() -> str:
    return os.environ.get("KBC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1507_02509_amd", "autotune.json"))


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(run, steps: int, reps: int) -> float:
    """Median milliseconds per step of run(steps) over reps repetitions."""
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run(steps)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    times.sort()
    return times[len(times) // 2]


def _model_key(params) -> list[str]:
    # the stabiliser mode and guard change the per-node cost (the exact root
    # runs a Newton iteration), so a choice made for one is not reused for another
    return [str(params.collision), str(params.variant), f"gm{params.gamma_mode}", f"guard{params.gamma_guard:.3e}"]


def _sim_key(sim) -> str:
    return "|".join(["sim3", torch.cuda.get_device_name(sim.device), str(sim.form), *_model_key(sim.params),
                     f"{sim.nx}x{sim.ny}"])


def tune_sim(sim, steps: int = 10, reps: int = 3, candidates=None, use_cache: bool = True):
    """Choose and apply the fastest launch configuration for this lattice;
    returns the chosen entry of STEP_CANDIDATES and the per-candidate
    timings."""
    path = cache_path()
    key = _sim_key(sim)
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        best = tuple(cache[key]["tile"])
        apply_config(sim, best)
        return best, cache[key].get("ms", {})
    steps += steps % 2
    snap = sim.state_buffer().clone()
    n0 = sim.steps
    timings = {}
    for cand in candidates or STEP_CANDIDATES:
        if cand[0] == "fused" and cand[1] == 32 and sim.form == _lib.F64:
            continue
        apply_config(sim, cand)
        sim.step(2)
        timings[cand] = _time(sim.step, steps, reps)
    best = min(timings, key=timings.get)
    apply_config(sim, best)
    sim.state_buffer().copy_(snap)
    sim.lib.lbm_set_step(sim.ctx, n0)
    torch.cuda.synchronize()
    if use_cache:
        cache = _load(path)
        cache[key] = {"tile": list(best), "ms": {str(list(k)): v for k, v in timings.items()}}
        _store(path, cache)
    return best, timings


def apply_ensemble_config(ens, cand):
    """Set a launch configuration from ENSEMBLE_CANDIDATES on an Ensemble."""
    if cand[0] == "single":
        ens.set_fusion(1)
        ens.set_tile(*cand[1:])
    else:
        ens.set_tile(256, 1, cand[2])
        ens.set_fusion(2, cand[1])


def _ens_key(ens) -> str:
    m0 = ens.members[0]
    sizes = hashlib.sha1(",".join(f"{m.nx}x{m.ny}" for m in ens.members).encode()).hexdigest()[:12]
    return "|".join(["ensemble3", torch.cuda.get_device_name(m0.device), str(m0.form), *_model_key(m0.params),
                     str(len(ens.members)), sizes])


def tune_ensemble(ens, steps: int = 10, reps: int = 3, persistent: bool = False, candidates=None,
                  use_cache: bool = True):
    """Choose and apply the fastest ensemble launch configuration; returns the
    chosen entry of ENSEMBLE_CANDIDATES and the timings."""
    path = cache_path()
    key = _ens_key(ens) + f"|{'persistent' if persistent else 'per-step'}"
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        best = tuple(cache[key]["tile"])
        apply_ensemble_config(ens, best)
        return best, cache[key].get("ms", {})
    steps += steps % 2
    snaps = [m.state_buffer().clone() for m in ens.members]
    n0 = [m.steps for m in ens.members]
    timings = {}
    for cand in candidates or ENSEMBLE_CANDIDATES:
        apply_ensemble_config(ens, cand)
        ens.step(2, persistent)
        timings[cand] = _time(lambda k: ens.step(k, persistent), steps, reps)
    best = min(timings, key=timings.get)
    apply_ensemble_config(ens, best)
    for m, snap, n in zip(ens.members, snaps, n0):
        m.state_buffer().copy_(snap)
        m.lib.lbm_set_step(m.ctx, n)
    torch.cuda.synchronize()
    if use_cache:
        cache = _load(path)
        cache[key] = {"tile": list(best), "ms": {str(list(k)): v for k, v in timings.items()}}
        _store(path, cache)
    return best, timings
