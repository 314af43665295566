"""Throughput of the hybrid SP-Shakhov / DSMC particle update on one MI355X.

Workload: the 2-D Ma 10 argon flow over a cylinder (Kn 0.01 on D, 800 x 600 cut-cell
grid, ~14.2M particles, diffuse wall at 500 K, freestream inflow on three sides), run
from the impulsive start for --warmup steps, then --steps timed steps with sampling on.
The headline runs the FP32-mixed path; the FP64 path is timed on the same workload for
the speed-up.  One step = the whole hot path: inflow, transport + walls, counting sort,
moments, time split, NTC DSMC, Shakhov resampling, conservation rescale, sampling.

Prints one JSON line.  `python bench.py --gpus N` with N > 1 exits: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the collide kernel (FP32-mixed, 2-D): per particle, the source index
# (4), the gathered source state x, y, vx, vy, vz, cell, id (32) and the written state (32);
# per cell, cell_start (4), volume (8), (sigma c)_max read + write (16) and, when sampling,
# the 13 FP64 sums read + written (208).
COLLIDE_BYTES_PER_PARTICLE = {"fp32": 68, "fp64": 4 + 64 + 64}
COLLIDE_BYTES_PER_CELL = 4 + 8 + 16 + 208


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(prec, case, gas, warmup, steps, graph_check=True):
    import torch
    from paper_2506_23917_amd.hs import Sim

    sim = Sim(gas, case, precision=prec, device="cuda:0")
    sim.set_timing(True)
    sim.step(warmup)
    sim.sync()
    warm_ms, warm_n = sim.kernel_timing("collide")
    sim.clear_timing()
    n0 = sim.num_particles(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n1 = sim.num_particles(0)
    res = dict(dt=dt, n0=n0, n1=n1)
    for k in ("inject", "move", "scan", "scatter", "collide", "step"):
        res[k + "_ms"] = sim.kernel_timing(k)[0]
    res["collide_ms_all"] = (warm_ms * warm_n + res["collide_ms"] * steps) / max(1, warm_n + steps)
    sim.clear_timing()
    sim.set_timing(False)
    return sim, res


def cpu_baseline(sim, case, gas, nsteps=1):
    """The FP64 oracle, single-threaded, on the GPU's developed state (imported), for
    nsteps steps; particle-steps / s."""
    import numpy as np
    from oracle.oracle import Oracle
    st = sim.export_state(0)
    ncell = st["cell"].astype(np.int64)
    nx, ny = case["nx"], case["ny"]
    x = np.zeros((len(ncell), 3))
    x[:, 0] = case["lo"][0] + (ncell % nx + st["pos"][:, 0].astype(np.float64)) * case["h"][0]
    x[:, 1] = case["lo"][1] + ((ncell // nx) % ny + st["pos"][:, 1].astype(np.float64)) * case["h"][1]
    ora = Oracle(gas, case)
    ora.set_state(0, x, st["vel"].astype(np.float64), st["cell"], st["id"], st["next_id"], st["step"])
    ora.set_cells(0, st["sigc_max"], st["acc"], st["n_samples"])
    n = ora.num_particles(0)
    t0 = time.perf_counter()
    ora.step(nsteps)
    dt = time.perf_counter() - t0
    return n * nsteps / dt, n, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--traffic", default=None, help="JSON file with rocprof FETCH/WRITE bytes per collide launch")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import workloads as W
    gas = W.gas()
    case = W.cylinder_2d()
    case["n_steady"] = args.warmup          # the timed steps sample (Step 5 is on)

    log("[bench] fp32-mixed: warmup %d, timed %d" % (args.warmup, args.steps))
    sim32, r32 = run_gpu("fp32", case, gas, args.warmup, args.steps)
    psteps = 0.5 * (r32["n0"] + r32["n1"]) * args.steps
    value = psteps / r32["dt"]
    ncells = case["nx"] * case["ny"]
    npart = 0.5 * (r32["n0"] + r32["n1"])
    sampling_cells = ncells
    coll_bytes = COLLIDE_BYTES_PER_PARTICLE["fp32"] * npart + COLLIDE_BYTES_PER_CELL * sampling_cells
    achieved = coll_bytes / (r32["collide_ms"] * 1e-3) / 1e9
    log("[bench] fp32: %.3f ms/step, %.3e particle-steps/s, collide %.3f ms" %
        (1e3 * r32["dt"] / args.steps, value, r32["collide_ms"]))

    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as f:
            t = json.load(f)
        traffic = t.get("bytes_per_launch")

    out = {
        "metric": "particle-steps/s, 2-D Ma10 cylinder: FP32-mixed vs FP64 at <=1e-3 moment error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["dt"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 moments, timescales, rescale)",
        "data": "synthetic",
        "config": {"workload": "2-D Ma10 argon cylinder, Kn 0.01 on D, 800x600 cut-cell grid, "
                               "~14.2M particles, FP32-mixed, steady sampling on",
                   "particles": int(npart), "cells": ncells},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "collide (wave + dense-cell launches)",
                     "kernel_ms": r32["collide_ms"], "kernel_ms_all_steps": r32["collide_ms_all"]},
        "kernels_ms": {k: r32[k + "_ms"] for k in ("inject", "move", "scan", "scatter", "collide", "step")},
    }
    if not args.no_fp64:
        del sim32
        import torch
        torch.cuda.empty_cache()
        log("[bench] fp64: warmup %d, timed %d" % (args.warmup, args.steps))
        sim64, r64 = run_gpu("fp64", case, gas, args.warmup, args.steps)
        v64 = 0.5 * (r64["n0"] + r64["n1"]) * args.steps / r64["dt"]
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["dt"] / args.steps,
                       "collide_ms": r64["collide_ms"]}
        out["mixed_speedup_vs_fp64"] = value / v64
        log("[bench] fp64: %.3f ms/step, %.3e particle-steps/s" % (1e3 * r64["dt"] / args.steps, v64))
        base_sim = sim64
    else:
        base_sim = sim32
    if not args.no_cpu:
        log("[bench] cpu oracle baseline")
        # the oracle takes FP64 state; the FP32 export is widened exactly
        v_cpu, n_cpu, t_cpu = cpu_baseline(base_sim, case, gas, args.cpu_steps)
        out["cpu_baseline"] = {"value": v_cpu, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": "%d step(s) of the same cylinder workload from the GPU's developed "
                                         "state after %d steps (%d particles, %.1f s)" %
                                         (args.cpu_steps, args.warmup + args.steps, n_cpu, t_cpu)}
        log("[bench] cpu: %.3e particle-steps/s (%.1f s)" % (v_cpu, t_cpu))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
