"""Benchmark of the cue-diffusion / growth-cone step on one MI355X.

A "step" is one time step of the whole hot path on the headline workload (2D 2048^2 FP32
field, 16 sources with rates U(0.5, 2), 65,536 growth cones, 1024 targets, D = 1, dt = 0.2,
k = 0.005): the stencil + decay + source update of every cell, then one gradient-sample /
turn / noise / advance / exit / contact step of every active cone.

Prints ONE JSON line:
  value          cell-updates per second over the K timed steps (inputs resident in HBM)
  roofline       the dominant kernel against the MI355X HBM peak (8 TB/s): algorithmic
                 bytes (8 B per cell-update: one FP32 read + one FP32 write) per launch /
                 average launch duration from HIP events on the library's stream
  cpu_baseline   the FP64 oracle on the host cores, on a bounded sample of the same
                 workload (rank 0, N = 1 only)
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

from paper_1405_3331_amd import binding as B  # noqa: E402
from paper_1405_3331_amd import scenarios as S  # noqa: E402

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_UPDATE = 8.0


def active_cone_steps(event_step, start, end):
    """Cone-steps performed in steps [start, end): a cone stopped at event step e did the
    steps 0 .. e-1; an active cone (e = -1) did every step."""
    e = np.where(event_step < 0, end, event_step).astype(np.int64)
    return int(np.clip(e, start, end).sum() - start * len(e))


def cpu_baseline(sc, steps):
    import oracle
    from oracle import build as obuild
    if not os.path.exists(oracle.LIBRARY):
        obuild.build()
    ref = oracle.OracleSim(sc)
    t0 = time.perf_counter()
    ref.step(steps)
    dt = time.perf_counter() - t0
    cone_steps = active_cone_steps(ref.event_step, 0, steps)
    return {
        "value": sc.n_cells * steps / dt,
        "unit": "cell-updates/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{sc.name}: first {steps} steps, all cells and cones (FP64, brute-force "
                  f"contact), {dt:.1f} s wall",
        "cone_steps_per_s": cone_steps / dt,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--block-steps", type=int, default=0,
                    help="steps per launch of the tiled kernel (0 = library default)")
    ap.add_argument("--cpu-steps", type=int, default=60,
                    help="steps of the oracle timed for cpu_baseline (0 = skip)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not "
              "supported (the single-GPU kernel is the unit of scaling)", file=sys.stderr)
        sys.exit(2)

    sc = S.headline()
    print(f"[bench] {sc.name}: {sc.n_cells} cells, {sc.n_cones} cones, "
          f"warmup {args.warmup}, timed {args.steps}", file=sys.stderr, flush=True)
    sim = B.Simulation(sc, block_steps=args.block_steps)
    tiling = sim.tiling()
    sim.step(args.warmup)
    sim.synchronize()
    if not args.no_kernel_timing:
        B.sim_set_timing(sim.h, True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.synchronize()
    elapsed = time.perf_counter() - t0
    ktime = B.sim_read_state(sim.h, B.KERNEL_TIME) if not args.no_kernel_timing else None
    c = sim.cones()
    cone_steps = active_cone_steps(c["event_step"], args.warmup, args.warmup + args.steps)
    sim.close()

    cells = sc.n_cells
    value = cells * args.steps / elapsed
    roofline = None
    if ktime is not None and ktime[1] > 0:
        launches = int(ktime[1])
        avg_ms = ktime[0] / launches
        steps_per_launch = args.steps / launches
        algo_bytes = BYTES_PER_CELL_UPDATE * cells * steps_per_launch
        achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "kernel_avg_us": avg_ms * 1e3, "launches": launches,
                    "steps_per_launch": steps_per_launch}
    out = {
        "metric": "cell-updates/s & cone-steps/s at 2048^2",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "grid": [sc.nx, sc.ny], "cones": sc.n_cones,
                   "targets": sc.n_targets, "sources": len(sc.species[0].source_q),
                   "D": sc.species[0].D, "k": sc.species[0].k, "dt": sc.dt,
                   "tiling": tiling},
        "cone_steps_per_s": cone_steps / elapsed,
        "active_cone_steps": cone_steps,
        "effective_GBs": value * BYTES_PER_CELL_UPDATE / 1e9,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
