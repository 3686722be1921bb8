"""Empirical autotuner for the tiled step kernel.

The library's planner picks the blocking depth B and the tile shape from a cost model.  This
module measures instead: for a scenario it times whole runs (the scenario's step count, so
that the late phase, when cones crowd around sources and targets, weighs in) of candidate
(B, row width, tile height) settings on the GPU through the C ABI -- on fresh copies of the
scenario, so nothing the caller holds is advanced -- and caches the fastest setting per size
class in ``tile_cache.json`` next to this file.  For a batch (one shared B and row width,
and a tile height hint for every simulation) it times batch launches per candidate and
records the fastest per batch class.

    python -m paper_1405_3331_amd.autotune headline      # tune and record a named workload
    python -m paper_1405_3331_amd.autotune batched       # the 512-simulation batch
"""
from __future__ import annotations

import copy
import json
import math
import os
import sys
import time

from . import binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tile_cache.json")


def size_class(sc) -> str:
    """Scenarios in one class share the best tiling: same grid, species count, step length
    in cells, and cone count within a factor of two."""
    cones = 0 if sc.n_cones == 0 else int(math.log2(sc.n_cones))
    return (f"{sc.dim}d:{sc.nx}x{sc.ny}x{sc.nz if sc.dim == 3 else 1}:"
            f"species{len(sc.species)}:step{sc.step_len / sc.dx:.3g}:cones2^{cones}")


def default_candidates():
    """(block_steps, cols_per_lane, height) triples; height 0 = the planner's choice.  The
    explicit heights keep two tiles resident per compute unit (LDS) at either row width;
    144 rows is the tallest 64 x 2-column tile that does."""
    return ([(b, 2, h) for b in (6, 8, 10, 12, 14, 16) for h in (0, 110, 130, 138, 144)] +
            [(b, 4, h) for b in (6, 8, 12, 16) for h in (0, 70)])


def _time_single(sc, block, cpl, height, steps):
    trial = copy.copy(sc)
    trial.tile = (cpl, height)
    sim = B.Simulation(trial, block_steps=block)
    tiling = sim.tiling()
    if tiling["block_steps"] != block:   # this depth does not fit the scenario
        sim.close()
        return None, tiling
    sim.step(block)                      # warm-up launch
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    dt = (time.perf_counter() - t0) / steps
    sim.close()
    return dt, tiling


def tune(sc, candidates=None, steps=None, verbose=False) -> dict:
    """Time every candidate (block_steps, cols_per_lane, height; 0 = planner's height) over
    `steps` steps (default: the scenario's run length) and return
    {"best": (block, cpl, height), "seconds_per_step": ..., "trials": [...]}."""
    steps = int(steps or getattr(sc, "n_steps", 0) or 2000)
    trials = []
    for block, cpl, height in candidates or default_candidates():
        dt, tiling = _time_single(sc, block, cpl, height, steps)
        trials.append({"block_steps": block, "cols_per_lane": cpl, "height": tiling["height"],
                       "seconds_per_step": dt})
        if verbose:
            print(f"[autotune] B={block} cpl={cpl} height={tiling['height']}: "
                  f"{'n/a' if dt is None else f'{dt * 1e6:.2f} us/step'}", flush=True)
    ok = [t for t in trials if t["seconds_per_step"] is not None]
    if not ok:
        raise RuntimeError("no candidate tiling fits this scenario")
    best = min(ok, key=lambda t: t["seconds_per_step"])
    return {"best": (best["block_steps"], best["cols_per_lane"], best["height"]),
            "seconds_per_step": best["seconds_per_step"], "trials": trials}


def batch_class(scenarios) -> str:
    """Batches in one class share the best launch shape: same simulation count and species
    count, total cells and total cones within a factor of two."""
    cells = sum(sc.n_cells for sc in scenarios)
    cones = sum(sc.n_cones for sc in scenarios)
    return (f"batch:{len(scenarios)}sims:species{len(scenarios[0].species)}:"
            f"cells2^{int(math.log2(max(cells, 1)))}:cones2^{int(math.log2(max(cones, 1)))}")


def default_batch_candidates():
    """(block_steps, cols_per_lane, height) for a batch: one shared depth and row width;
    height is every simulation's tile height hint (0 = each simulation's planner)."""
    return ([(b, 2, h) for b in (4, 6, 8, 10, 12, 16) for h in (0, 110)] +
            [(b, 4, 0) for b in (6, 8, 12)])


def _with_tile(scenarios, cpl, height):
    out = []
    for sc in scenarios:
        trial = copy.copy(sc)
        trial.tile = (cpl, height)
        out.append(trial)
    return out


def tune_batch(scenarios, candidates=None, launches=8, verbose=False) -> dict:
    """Time batch launches (persistent grid, no graph) of every candidate (block_steps,
    cols_per_lane, height) over `launches` full-depth launches; return
    {"best": (block, cpl, height), "seconds_per_step": ..., "trials": [...]}."""
    trials = []
    cells = sum(sc.n_cells for sc in scenarios)
    for block, cpl, height in candidates or default_batch_candidates():
        try:
            bt = B.Batch(_with_tile(scenarios, cpl, height), graph_launches=0,
                         block_steps=block)
        except B.SimError:
            trials.append({"block_steps": block, "cols_per_lane": cpl, "height": height,
                           "seconds_per_step": None})
            continue
        bt.step(block)
        bt.synchronize()
        t0 = time.perf_counter()
        bt.step(block * launches)
        bt.synchronize()
        dt = (time.perf_counter() - t0) / (block * launches)
        bt.close()
        trials.append({"block_steps": block, "cols_per_lane": cpl, "height": height,
                       "seconds_per_step": dt})
        if verbose:
            print(f"[autotune] batch B={block} cpl={cpl} height={height}: "
                  f"{dt * 1e6:.1f} us/step, {cells / dt:.3e} cell-updates/s", flush=True)
    ok = [t for t in trials if t["seconds_per_step"] is not None]
    if not ok:
        raise RuntimeError("no candidate launch shape fits this batch")
    best = min(ok, key=lambda t: t["seconds_per_step"])
    return {"best": (best["block_steps"], best["cols_per_lane"], best["height"]),
            "seconds_per_step": best["seconds_per_step"], "trials": trials}


def record_batch(scenarios, result, path=CACHE):
    cache = load_cache(path)
    cache[batch_class(scenarios)] = {
        "block_steps": result["best"][0], "cols_per_lane": result["best"][1],
        "height": result["best"][2], "seconds_per_step": result["seconds_per_step"]}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def apply_batch(scenarios, path=CACHE) -> int:
    """Set every scenario's tile hint from the batch class's record; return the shared
    block_steps (0 when the class was never tuned: the library default)."""
    hit = load_cache(path).get(batch_class(scenarios))
    if not hit:
        return 0
    for sc in scenarios:
        sc.tile = (hit["cols_per_lane"], hit["height"])
    return hit["block_steps"]


def load_cache(path=CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def record(sc, result, path=CACHE):
    cache = load_cache(path)
    cache[size_class(sc)] = {"block_steps": result["best"][0], "cols_per_lane": result["best"][1],
                             "height": result["best"][2],
                             "seconds_per_step": result["seconds_per_step"]}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def lookup(sc, path=CACHE):
    """(block_steps, cols_per_lane, height) recorded for the scenario's size class, or None."""
    hit = load_cache(path).get(size_class(sc))
    if not hit:
        return None
    return hit["block_steps"], hit["cols_per_lane"], hit["height"]


def apply(sc, path=CACHE) -> int:
    """Set the scenario's tile hint from the cache; return the block_steps to use (0 when
    the size class was never tuned: the library's planner decides)."""
    hit = lookup(sc, path)
    if hit is None:
        return 0
    sc.tile = (hit[1], hit[2])
    return hit[0]


def main(argv):
    from . import scenarios
    names = argv or ["headline"]
    for name in names:
        if name == "batched":
            scs = scenarios.batched()
            print(f"[autotune] batched ({batch_class(scs)})", flush=True)
            res = tune_batch(scs, verbose=True)
            record_batch(scs, res)
        else:
            sc = scenarios.NAMED[name]()
            print(f"[autotune] {sc.name} ({size_class(sc)})", flush=True)
            res = tune(sc, verbose=True)
            record(sc, res)
        print(f"[autotune] best {res['best']} at {res['seconds_per_step'] * 1e6:.2f} us/step",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
