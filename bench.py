"""Benchmark of the cue-diffusion / growth-cone step on one MI355X.

A "step" is one time step of the whole hot path on the headline workload (2D 2048^2 FP32
field, 16 sources with rates U(0.5, 2), 65,536 growth cones, 1024 targets, D = 1, dt = 0.2,
k = 0.005): the stencil + decay + source update of every cell, then one gradient-sample /
turn / noise / advance / exit / contact step of every active cone.

Prints ONE JSON line:
  value             cell-updates per second over the K timed steps (inputs resident in HBM)
  cone_steps_per_s  active cone-steps of the K steps / (their HIP-event time - the time of
                    the same K steps of the same field with no cones and no targets)
  roofline          the dominant kernel against the MI355X HBM peak (8 TB/s): algorithmic
                    bytes (8 B per cell-update: one FP32 read + one FP32 write) per launch /
                    average launch duration from HIP events on the library's stream
  batched_vs_plain  512 uneven simulations in one persistent launch per block (hipGraph,
                    autotuned launch shape) against the same simulations one at a time
  adjoint_vs_plain  the 1024^2 trajectory-loss gradient (checkpointed forward + reverse
                    sweep) against the plain forward run of the same steps
  cpu_baseline      the FP64 oracle on the host cores, on a bounded sample of the same
                    workload (rank 0, N = 1 only)
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1405_3331_amd import autotune  # noqa: E402
from paper_1405_3331_amd import binding as B  # noqa: E402
from paper_1405_3331_amd import scenarios as S  # noqa: E402

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_UPDATE = 8.0
# Counter-derived HBM traffic of the step kernel, recorded from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs; used only while the kernel sources still hash to the recorded value.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "tiled_step_headline_2048_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1405_3331_amd", "csrc", f)
                  for f in ("kernels_tiled.hip", "device.hpp", "tiled.hpp", "internal.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(tiling):
    """HBM bytes per launch from the committed counter record, or None when the record is
    missing, was taken for another tiling, or the kernel sources changed since."""
    try:
        rec = dict(line.strip().split("=", 1) for line in open(TRAFFIC_RECORD)
                   if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    if rec.get("tiling") != json.dumps(tiling, sort_keys=True):
        return None
    return float(rec["hbm_bytes_per_launch"])


def copy_calibration(mbytes):
    """Device-to-device copy of a known size (the runtime's blit kernel), for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    n = int(mbytes) << 20
    src, dst = C.c_void_p(), C.c_void_p()
    assert hip.hipMalloc(C.byref(src), C.c_size_t(n)) == 0
    assert hip.hipMalloc(C.byref(dst), C.c_size_t(n)) == 0
    assert hip.hipMemset(src, 1, C.c_size_t(n)) == 0
    for _ in range(3):
        assert hip.hipMemcpy(dst, src, C.c_size_t(n), 3) == 0   # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(src)
    hip.hipFree(dst)
    print(f"[bench] copy calibration: 3 x {n} bytes device to device", file=sys.stderr,
          flush=True)


def active_cone_steps(event_step, start, end):
    """Cone-steps performed in steps [start, end): a cone stopped at event step e did the
    steps 0 .. e-1; an active cone (e = -1) did every step."""
    e = np.where(event_step < 0, end, event_step).astype(np.int64)
    return int(np.clip(e, start, end).sum() - start * len(e))


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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
        "host": host_cpu_model(),
        "kind": "oracle",
        "sample": f"{sc.name}: first {steps} steps, all cells and cones (FP64, brute-force "
                  f"contact), {dt:.1f} s wall",
        "cone_steps_per_s": cone_steps / dt,
    }


def measure_batched(steps, graph_launches, count=512):
    """512 uneven simulations: one persistent launch per block of steps (hipGraph replay, the
    depth, row width and tile height the autotuner recorded for this batch class) against
    the same simulations advanced one after another through sim_step (each simulation's
    library default).  Inputs are resident on the device before either timed region."""
    scs = S.batched(count=count)
    cells = sum(sc.n_cells for sc in scs)
    block = autotune.apply_batch(scs)
    print(f"[bench] batched: {len(scs)} simulations, {cells} cells, {steps} steps, "
          f"block_steps {block or 'default'}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    bt = B.Batch(scs, graph_launches=graph_launches, block_steps=block)
    create_s = time.perf_counter() - t0
    bt.step(graph_launches * 8 if graph_launches else 8)   # warm-up
    bt.synchronize()
    t0 = time.perf_counter()
    bt.step(steps)
    bt.synchronize()
    batched_s = time.perf_counter() - t0
    t0_tiling = bt.tiling(0)
    tiling = {"block_steps": t0_tiling["block_steps"],
              "cols_per_lane": t0_tiling["cols_per_lane"],
              "height_hint": int((getattr(scs[0], "tile", None) or (0, 0))[1])}
    bt.close()
    # the same simulations one at a time (library default path per simulation)
    sims = [B.Simulation(sc) for sc in S.batched(count=count)]
    for sim in sims:
        sim.step(8)
    for sim in sims:
        sim.synchronize()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(steps)
    for sim in sims:
        sim.synchronize()
    single_s = time.perf_counter() - t0
    for sim in sims:
        sim.close()
    return {
        "value": cells * steps / batched_s,
        "plain_value": cells * steps / single_s,
        "batched_over_plain": single_s / batched_s,
        "steps": steps, "cells": cells, "cones": sum(sc.n_cones for sc in scs),
        "graph_launches": graph_launches, "tiling": tiling, "create_s": create_s,
    }


def bench_batched(args):
    m = measure_batched(args.batch_steps, args.graph_launches, args.batch_count)
    out = {
        "metric": "batched cell-updates/s vs one simulation at a time (same GPU)",
        "value": m["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": m["steps"], "higher_is_better": True, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched {args.batch_count} 2D simulations, side U{{64..512}}, "
                               "cones log-uniform [16, 4096]", "cells": m["cells"],
                   "cones": m["cones"], "graph_launches": m["graph_launches"],
                   "tiling": m["tiling"]},
        "one_at_a_time_value": m["plain_value"],
        "speedup_vs_one_at_a_time": m["batched_over_plain"],
        "effective_GBs": m["value"] * BYTES_PER_CELL_UPDATE / 1e9,
        "create_s": m["create_s"],
    }
    print(json.dumps(out), flush=True)


def measure_adjoint(steps, every):
    """Gradient of the trajectory loss sum_i |p_i^N - t_(i mod 256)|^2 of the 2D 1024^2
    workload (32 sources, 8192 cones) with respect to the 32 source amounts, D and k: the
    checkpointed forward run plus the reverse sweep, against the plain forward run of the
    same steps on the same GPU."""
    sc = S.adjoint()
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]
    weight = np.ones(M)
    print(f"[bench] {sc.name}: {sc.n_cells} cells, {M} cones, {steps} steps, checkpoint "
          f"every {every}", file=sys.stderr, flush=True)
    block = autotune.apply(sc)
    sim = B.Simulation(sc, block_steps=block)
    sim.step(16)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    forward_s = time.perf_counter() - t0
    sim.close()
    # warm-up: a short gradient run loads the reverse-sweep kernels (code objects load on
    # first launch)
    sim = B.Simulation(sc, block_steps=block)
    sim.adjoint(2 * every, assign, weight, every)
    sim.adjoint_backward()
    sim.close()
    sim = B.Simulation(sc, block_steps=block)
    t0 = time.perf_counter()
    loss = sim.adjoint(steps, assign, weight, every)
    t1 = time.perf_counter()
    dq, dD, dk = sim.adjoint_backward()
    t2 = time.perf_counter()
    sim.close()
    grad_s = t2 - t0
    return {
        "value": sc.n_cells * steps / grad_s, "plain_value": sc.n_cells * steps / forward_s,
        "gradient_over_forward": grad_s / forward_s, "steps": steps, "checkpoint_every": every,
        "forward_s": forward_s, "adjoint_forward_s": t1 - t0, "reverse_s": t2 - t1,
        "loss": loss, "dL_dD": float(dD[0]), "dL_dk": float(dk[0]),
        "dL_dq_norm": float(np.linalg.norm(dq)),
    }


def bench_adjoint(args):
    m = measure_adjoint(args.adjoint_steps, args.checkpoint_every)
    out = {
        "metric": "adjoint (trajectory-loss gradient) cell-updates/s vs the plain forward run",
        "value": m["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": m["steps"], "higher_is_better": True, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "adjoint 2D 1024^2, 32 sources, 8192 cones, 256 targets, "
                               "loss sum |p_i - t_(i mod 256)|^2",
                   "checkpoint_every": m["checkpoint_every"]},
    }
    out.update({k: v for k, v in m.items() if k not in ("value", "steps", "checkpoint_every")})
    print(json.dumps(out), flush=True)


# SNR turn law parameters of the --snr run: snr_scale, cone_width, kd, c_min, c_max
SNR_LAW = (50.0, 1.0, 0.5, 1e-3, 1e3)


def bench_connectivity(args):
    """The connections of the headline run after --connectivity-steps steps: the adjacency
    list (V_a, E_a) of neuron -> neuron contacts and the BFS levels from neuron 0 (Sec. 3.4,
    Figs. 4-5), 16 cones per neuron (65,536 cones -> 4096 neurons), targets owned by a fixed
    affine map.  Times each call end to end (host arrays in and out)."""
    sc = S.headline()
    steps = args.connectivity_steps
    n_neurons = sc.n_cones // 16
    cone_owner = np.arange(sc.n_cones) // 16
    target_owner = (np.arange(sc.n_targets) * 7 + 3) % n_neurons
    block = autotune.apply(sc)
    sim = B.Simulation(sc, block_steps=block)
    sim.step(steps)
    sim.synchronize()
    sim.connectivity(n_neurons, cone_owner, target_owner)   # warm-up (first launches)
    sim.bfs_levels(0, n_neurons)
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        row_start, edges = sim.connectivity(n_neurons, cone_owner, target_owner)
    t1 = time.perf_counter()
    for _ in range(reps):
        level = sim.bfs_levels(0, n_neurons)
    t2 = time.perf_counter()
    counts = sim.counts()
    sim.close()
    conn_ms = (t1 - t0) * 1e3 / reps
    out = {
        "metric": "connectivity: adjacency list and BFS levels of the contacts, ms per call",
        "value": conn_ms, "unit": "ms", "n_gpus": 1, "higher_is_better": False,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{sc.name} after {steps} steps, 16 cones per neuron",
                   "neurons": n_neurons, "cones": sc.n_cones, "targets": sc.n_targets},
        "edges": int(edges.size), "contacts": int(counts[1]),
        "adjacency_ms": conn_ms, "bfs_ms": (t2 - t1) * 1e3 / reps,
        "bfs_depth": int(level.max()), "reached": int((level >= 0).sum()),
    }
    print(json.dumps(out), flush=True)


def bench_volume(args):
    """3D 256^3 two-species workload through the per-step path (one stencil + sources launch
    for both species, then one thread per cone in spatial order)."""
    sc = S.volume()
    ns = len(sc.species)
    steps = args.volume_steps
    print(f"[bench] {sc.name}: {sc.n_cells} cells x {ns} species, {sc.n_cones} cones, "
          f"{steps} steps", file=sys.stderr, flush=True)
    sim = B.Simulation(sc)
    sim.step(10)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    elapsed = time.perf_counter() - t0
    c = sim.cones()
    cone_steps = active_cone_steps(c["event_step"], 10, 10 + steps)
    # the stencil kernel's own duration, from a further stretch of steps whose field
    # launches each record a pair of events (outside the timed region: the events add
    # several microseconds of dispatch gap per launch)
    B.sim_set_timing(sim.h, True)
    sim.step(min(steps, 100))
    sim.synchronize()
    ktime = B.sim_read_state(sim.h, B.KERNEL_TIME)
    sim.close()
    updates = sc.n_cells * ns * steps
    avg_us = ktime[0] / ktime[1] * 1e3
    # one launch per step covers the stencil and sources of every species
    achieved = BYTES_PER_CELL_UPDATE * sc.n_cells * ns / (avg_us * 1e-6) / 1e9
    out = {
        "metric": "species-cell-updates/s & cone-steps/s, 3D 256^3 two species",
        "value": updates / elapsed, "unit": "species-cell-updates/s", "n_gpus": 1,
        "steps": steps, "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": sc.name, "grid": [sc.nx, sc.ny, sc.nz], "species": ns,
                   "cones": sc.n_cones, "targets": sc.n_targets},
        "cone_steps_per_s": cone_steps / elapsed,
        "roofline": {"bound": "hbm", "kernel": "stencil + sources (all species, one step)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "kernel_avg_us": avg_us},
    }
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(sc, max(1, args.cpu_steps // 10))
    print(json.dumps(out), flush=True)


def without_cones(sc):
    """The same scenario with no cones and no targets (the field update alone)."""
    bare = copy.copy(sc)
    bare.cone_pos = sc.cone_pos[:0]
    bare.cone_dir = sc.cone_dir[:0]
    bare.target_pos = sc.target_pos[:0]
    return bare


def timing_events(stream):
    """A pair of timing events on `stream`, recorded once and followed by a synchronize of the
    stream: the first stream synchronize after an event record on a stream costs about 20 us
    more than later ones (measured in fresh processes on the 20-step headline region), a
    one-time cost that would otherwise land inside the timed region."""
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    ev1.record(stream)
    stream.synchronize()
    return ev0, ev1


def timed_region(sc, stream, block, warmup, steps):
    """HIP-event milliseconds of `steps` steps of `sc` after `warmup` steps, on `stream`,
    and the tiling used."""
    sim = B.Simulation(sc, stream=stream, block_steps=block)
    tiling = sim.tiling()
    sim.step(warmup)
    sim.synchronize()
    ev0, ev1 = timing_events(stream)
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    sim.synchronize()
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    sim.close()
    return ms, tiling


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--block-steps", type=int, default=0,
                    help="steps per launch of the tiled kernel (0 = the autotuner's record "
                         "for this workload, else the library default)")
    ap.add_argument("--cpu-steps", type=int, default=600,
                    help="steps of the oracle timed for cpu_baseline, about 10 s of the "
                         "host's cores on the headline workload (0 = skip)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run a device-to-device copy of this size first (for counters)")
    ap.add_argument("--batched", action="store_true",
                    help="measure the batched workload instead of the headline one")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--graph-launches", type=int, default=10)
    ap.add_argument("--volume", action="store_true",
                    help="measure the 3D two-species workload instead of the headline one")
    ap.add_argument("--volume-steps", type=int, default=400)
    ap.add_argument("--adjoint", action="store_true",
                    help="measure the trajectory-loss gradient of the 1024^2 workload")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--checkpoint-every", type=int, default=100)
    ap.add_argument("--snr", action="store_true",
                    help="the headline workload under the SNR turn law (Sec. 3.5, Eq. 5)")
    ap.add_argument("--connectivity", action="store_true",
                    help="adjacency list and BFS levels of the headline run's contacts")
    ap.add_argument("--connectivity-steps", type=int, default=4000)
    ap.add_argument("--stencil-only", action="store_true",
                    help="the headline grid with no cones and no targets (field update only)")
    ap.add_argument("--call-steps", type=int, default=0,
                    help="step the timed region in calls of this many steps, one launch each "
                         "when it is at most the blocking depth (0 = one call)")
    ap.add_argument("--no-cone-rate", action="store_true",
                    help="skip the stencil-only run behind cone_steps_per_s")
    ap.add_argument("--ratio-batch-steps", type=int, default=400,
                    help="steps of the batched-vs-plain comparison on the default line "
                         "(0 = skip)")
    ap.add_argument("--ratio-adjoint-steps", type=int, default=2000,
                    help="steps of the adjoint-vs-plain comparison on the default line "
                         "(0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not "
              "supported (the single-GPU kernel is the unit of scaling)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration_mb > 0:
        copy_calibration(args.copy_calibration_mb)
    if args.batched:
        bench_batched(args)
        return
    if args.volume:
        bench_volume(args)
        return
    if args.adjoint:
        bench_adjoint(args)
        return
    if args.connectivity:
        bench_connectivity(args)
        return
    sc = S.headline()
    if args.snr:
        sc.snr_law = SNR_LAW
        sc.name += ", SNR turn law"
    block = args.block_steps
    if block == 0:   # blocking depth and tile shape recorded by the autotuner, if any
        block = autotune.apply(sc)
    if args.stencil_only:   # after the lookup: the tiling stays the headline's
        sc = without_cones(sc)
        sc.name += ", stencil only"
        args.no_cone_rate = True
    print(f"[bench] {sc.name}: {sc.n_cells} cells, {sc.n_cones} cones, "
          f"warmup {args.warmup}, timed {args.steps}, block_steps {block or 'default'}",
          file=sys.stderr, flush=True)
    # The library's launches go on a stream of ours, so that one pair of HIP events on it
    # brackets exactly the timed launches (no event between launches perturbs them).
    import torch
    stream = torch.cuda.Stream()
    sim = B.Simulation(sc, stream=stream, block_steps=block)
    tiling = sim.tiling()
    sim.step(args.warmup)
    sim.synchronize()
    ev0, ev1 = timing_events(stream)
    ev0.record(stream)
    t0 = time.perf_counter()
    if args.call_steps > 0:
        for done in range(0, args.steps, args.call_steps):
            sim.step(min(args.call_steps, args.steps - done))
    else:
        sim.step(args.steps)
    ev1.record(stream)
    sim.synchronize()
    elapsed = time.perf_counter() - t0
    ev1.synchronize()
    gpu_ms = ev0.elapsed_time(ev1)
    c = sim.cones()
    cone_steps = active_cone_steps(c["event_step"], args.warmup, args.warmup + args.steps)
    sim.close()
    # cone-steps/s as active cone-steps / (t_with_cones - t_stencil_only): the same steps of
    # the same field with no cones and no targets, in the same tiling, on HIP event time
    cone_rate = None
    if not args.no_cone_rate:
        bare = without_cones(sc)
        bare_ms, bare_tiling = timed_region(bare, stream, block, args.warmup, args.steps)
        extra_ms = gpu_ms - bare_ms
        cone_rate = {
            "value": cone_steps / (extra_ms * 1e-3) if extra_ms > 0 else None,
            "unit": "cone-steps/s", "active_cone_steps": cone_steps,
            "with_cones_ms": gpu_ms, "stencil_only_ms": bare_ms,
            "same_tiling": bare_tiling == tiling,
        }

    cells = sc.n_cells
    value = cells * args.steps / elapsed
    roofline = None
    block_used = max(1, tiling["block_steps"])
    launches = -(-args.steps // block_used)   # the tiled kernel's launches in the region
    if not args.no_kernel_timing and tiling["block_steps"] > 1:
        # the timed region holds only the step kernel's launches: their average duration
        # (back-to-back dispatch gaps included) is the region's event time over the count
        avg_ms = gpu_ms / launches
        steps_per_launch = args.steps / launches
        algo_bytes = BYTES_PER_CELL_UPDATE * cells * steps_per_launch
        achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
        # the counter record was taken under the vector-addition law
        traffic = recorded_traffic(tiling) if tiling["block_steps"] > 1 and not args.snr else None
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
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
        "cone_steps_per_s": cone_rate["value"] if cone_rate else None,
        "cone_rate": cone_rate,
        "effective_GBs": value * BYTES_PER_CELL_UPDATE / 1e9,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.snr:
        # the second half of the metric: batched and adjoint throughput against the plain
        # per-simulation path on the same GPU (short runs of those workloads)
        if args.ratio_batch_steps > 0:
            m = measure_batched(args.ratio_batch_steps, args.graph_launches)
            out["batched_vs_plain"] = {
                "workload": "512 uneven 2D simulations, one persistent launch per block "
                            "(hipGraph) vs sim_step per simulation",
                "steps": m["steps"], "batched_cell_updates_per_s": m["value"],
                "plain_cell_updates_per_s": m["plain_value"],
                "ratio": m["batched_over_plain"], "tiling": m["tiling"]}
        if args.ratio_adjoint_steps > 0:
            m = measure_adjoint(args.ratio_adjoint_steps, args.checkpoint_every)
            out["adjoint_vs_plain"] = {
                "workload": "2D 1024^2 trajectory-loss gradient (32 q, D, k), checkpoint "
                            f"every {m['checkpoint_every']}, vs the plain forward run",
                "steps": m["steps"], "gradient_s": m["adjoint_forward_s"] + m["reverse_s"],
                "forward_s": m["forward_s"], "ratio": m["gradient_over_forward"]}
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
