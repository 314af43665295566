"""Throughput of the hybrid SP-Shakhov / DSMC particle update on one MI355X.

Workload: the 2-D Ma 10 argon flow over a cylinder (Kn 0.01 on D, 800 x 600 cut-cell grid,
~14.2M particles, diffuse wall at 500 K, freestream inflow on three sides, vacuum outflow),
run from the impulsive start for --warmup steps, then --steps timed steps with sampling on.
The headline runs the FP32-mixed path; the FP64 path is timed on the same workload for the
speed-up.  One step = the whole hot path: inflow, transport + walls, counting sort, moments,
time split, NTC DSMC, Shakhov resampling, conservation rescale, sampling.  Inputs are
resident in HBM when the timed region starts (the state never leaves the device).

The roofline object is for the dominant kernel (the tile collision kernel), timed with HIP
events on the simulation's stream inside the timed region.  Its HBM traffic is the ratio of
counter bytes to algorithmic bytes from a committed rocprofv3 counter summary times the
algorithmic bytes of the timed state, reported only while the kernel sources are the ones
it was measured on; so is `valu_active_frac`, the share of the kernel's time its SIMDs
spend issuing vector-ALU instructions (SQ counters), which shows what bounds it instead of HBM.

The FP64 run's developed state is then imported into an FP32-mixed sim and both take one step
from it with the same random numbers: the relative L2 differences of the cell moments n, u, T, q
go into the line's "accuracy" object (the mixed path's bound is 1e-3).

`--workload ogrid` measures the body-fitted mesh path instead: a batch of twelve O-grid runs of
the paper's Ma 5 cylinder (first layer 1 mm, growth 1.1 or 1.05, Kn 0.01 or 0.1; ~10.4M
particles, 149k quads), face-to-face tracking in k_move_mesh.  `--workload sphere_hex` the
Ma 10 sphere of Sec. 4.4 on a 72 x 36 x 76 hexahedral shell (197k cells, ~6M particles).  Their
roofline object is for the move group (k_move_fast passing the mesh waves + k_move_mesh), timed
the same way.

Prints one JSON line.  `python bench.py --gpus N` with N > 1 exits: the build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one launch of the tile collision kernel (FP32-mixed): per particle,
# its velocity read and written (12 + 12); per cell, cell_start (4), the scalar record
# U, T, P_relax, (sigma c)_max, N_col, flags (64), (sigma c)_max written (8) and the 13 FP64
# sampling sums read and written (208).
TILE_BYTES_PER_PARTICLE = 24
TILE_BYTES_PER_CELL = 4 + 64 + 8 + 208
# Whole step, FP32-mixed 2-D: one state read + write for the sort and one for move and
# collide, plus cell traffic (about 128 B per particle-step).
STEP_BYTES_PER_PARTICLE = 128
# Mesh move (FP32-mixed, per particle): cell (4), position (8) and velocity (12) read;
# position, velocity, new cell and slot written (8 + 12 + 4 + 4).  Node coordinates and
# neighbours are per cell and stay in cache.
MESH_MOVE_BYTES_PER_PARTICLE = 24 + 28
HEX_MOVE_BYTES_PER_PARTICLE = 28 + 32      # the same in 3-D: 4 + 12 + 12 read, 12 + 12 + 4 + 4 written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "collide_tile_cylinder_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "collide_tile_cylinder_valu.txt")
STEP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cylinder_step_traffic.md")
# HIP timing events go into every TIMING_PERIOD-th timed step only: each event costs the
# stream a few microseconds, and the kernel's average is taken over launches spread evenly
# through the timed region.
TIMING_PERIOD = 8
KERNEL_SOURCES = ["hs_kernels.hip", "hs_device.hpp", "hs_common.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2506_23917_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _committed_value(path, key):
    """A `key: value` figure of a committed counter summary, if the summary was measured on
    the current kernel sources (its kernel_source_sha256 line); else None."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    m_v = re.search(re.escape(key) + r":\s*([0-9.eE+]+)", txt)
    if not m_h or not m_v or m_h.group(1) != kernel_source_hash():
        return None
    return float(m_v.group(1))


def committed_traffic_ratio():
    """HBM bytes over algorithmic bytes of the tile kernel from the committed counter summary,
    if it was measured on the current kernel sources; else None.  The bench multiplies it by
    the algorithmic bytes of the state it times, so the traffic it reports is that state's."""
    return _committed_value(TRAFFIC_FILE, "hbm_traffic_over_algorithmic")


def committed_valu():
    """Share of the tile kernel's time its SIMDs spend issuing VALU instructions, from the
    committed SQ counter summary, if it was measured on the current kernel sources; else None."""
    return _committed_value(VALU_FILE, "valu_active_frac")


def committed_step_bytes():
    """HBM bytes per particle-step of the whole cylinder step by the counters of every kernel
    (the committed summary), if measured on the current kernel sources; else None."""
    return _committed_value(STEP_TRAFFIC_FILE, "step_hbm_bytes_per_particle_step")


def step_roofline(value):
    """The whole step against the HBM peak: at the planned 128 B per particle-step, and at the
    bytes every kernel of the step moves by the committed counter summary (None if that
    summary was measured on other kernel sources)."""
    out = {"bytes_per_particle_step": STEP_BYTES_PER_PARTICLE,
           "achieved_GBs": STEP_BYTES_PER_PARTICLE * value / 1e9,
           "frac": STEP_BYTES_PER_PARTICLE * value / 1e9 / HBM_PEAK_GBS}
    b = committed_step_bytes()
    out["counter_bytes_per_particle_step"] = b
    out["counter_achieved_GBs"] = b * value / 1e9 if b else None
    out["counter_frac"] = b * value / 1e9 / HBM_PEAK_GBS if b else None
    return out


def host_cpu():
    """CPU model and logical CPU counts of this host (for the CPU baseline's record)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def run_gpu(prec, case, gas, warmup, steps, timed_group="collide", develop=0):
    import torch
    from paper_2506_23917_amd.hs import Sim

    sim = Sim(gas, case, precision=prec, device="cuda:0")
    if develop:
        sim.step(develop)
    sim.step(warmup)
    sim.sync()
    # launch shapes (blocks per grid of each kernel group) picked by the autotuner on the
    # developed flow; its trial steps are further warmup steps
    tune = sim.autotune(steps_per_trial=10)
    nc = len(sim.cases)
    n0 = sum(sim.num_particles(c) for c in range(nc))
    sim.set_timing([timed_group], period=TIMING_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n1 = sum(sim.num_particles(c) for c in range(nc))
    tile_ms, launches = sim.kernel_timing(timed_group)
    sim.set_timing(False)
    sim.clear_timing()
    return sim, dict(dt=dt, n0=n0, n1=n1, tile_ms=tile_ms, launches=launches, tune=tune,
                     before=develop + warmup + tune["steps"])


def membership(st, ncells):
    """Per cell: particle count and a wrapping 64-bit sum of hashed ids (equal in two states
    exactly when the cell holds the same particles, up to hash collisions)."""
    import numpy as np
    cell = st["cell"].astype(np.int64)
    h = st["id"].astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    cnt = np.bincount(cell, minlength=ncells)
    starts = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    hs = np.zeros(ncells, np.uint64)
    nz = cnt > 0
    if nz.any():
        hs[nz] = np.add.reduceat(h, starts[nz])
    return cnt, hs


def paired_accuracy(sim64, case, gas):
    """FP32-mixed against FP64 from the same developed state and RNG stream: one step of each,
    relative L2 over the cells of n, T and q, and of u relative to the local speed scale
    sqrt(|u|^2 + kT/m).  A particle that FP32 rounding puts in the neighbouring cell changes
    that cell's NTC pairs, so the figure is also given over the cells that hold the same
    particles in both runs (the precision error proper) with the number of cells that do
    not, and beside it the same measure for an FP64 step from the same state with another
    seed (the statistical noise of the current-state moments after one step)."""
    import numpy as np
    from paper_2506_23917_amd.hs import Sim
    st = sim64.export_state(0)
    s32 = Sim(gas, case, precision="fp32", device="cuda:0", no_particles=True)
    s32.import_state(0, st)
    s32.step(1)
    s64b = Sim(gas, dict(case, seed=case["seed"] + 976), precision="fp64", device="cuda:0", no_particles=True)
    s64b.import_state(0, st)
    s64b.step(1)
    sim64.step(1)
    del st
    a, b, c = s32.sample_moments(0, mode=1), sim64.sample_moments(0, mode=1), s64b.sample_moments(0, mode=1)
    nc = len(b["n"])
    m32, m64 = membership(s32.export_state(0), nc), membership(sim64.export_state(0), nc)
    occupied = b["n"] > 0
    same = occupied & (m32[0] == m64[0]) & (m32[1] == m64[1])

    def l2(x, y, sel):
        out = {k: float(np.sqrt(np.sum((x[k][sel] - y[k][sel]) ** 2)) / max(np.sqrt(np.sum(y[k][sel] ** 2)), 1e-300))
               for k in ("n", "T", "q")}
        scale = np.sqrt(np.sum(y["u"][sel] ** 2) + np.sum(1.380649e-23 * np.maximum(y["T"][sel], 0.0) / gas["m"]))
        out["u"] = float(np.sqrt(np.sum((x["u"][sel] - y["u"][sel]) ** 2)) / scale)
        return out

    out = dict(all_cells=l2(a, b, occupied), same_particles=l2(a, b, same),
               cells_with_other_particles=int(np.sum(occupied & ~same)), occupied_cells=int(np.sum(occupied)),
               fp64_other_seed=l2(c, b, occupied))
    del s32, s64b
    return out


def cpu_baseline(sim, case, gas, nsteps):
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


def main_ogrid(args):
    """A body-fitted mesh workload (the O-grid batch or the hexahedral sphere): FP32-mixed and
    FP64 throughput, the mesh move kernels against the HBM roofline."""
    import workloads as W
    gas = W.gas()
    hexa = args.workload == "sphere_hex"
    cases = [W.sphere_hex()] if hexa else W.ogrid_batch()
    for c in cases:
        c["n_steady"] = args.warmup
    ncells = sum(len(c["mesh"]["quad"]) for c in cases)
    log("[bench] %s fp32-mixed: warmup %d, timed %d" % (args.workload, args.warmup, args.steps))
    sim32, r32 = run_gpu("fp32", cases, gas, args.warmup, args.steps, timed_group="move")
    npart = 0.5 * (r32["n0"] + r32["n1"])
    value = npart * args.steps / r32["dt"]
    ms_step = 1e3 * r32["dt"] / args.steps
    move_bytes = (HEX_MOVE_BYTES_PER_PARTICLE if hexa else MESH_MOVE_BYTES_PER_PARTICLE) * npart
    achieved = move_bytes / (r32["tile_ms"] * 1e-3) / 1e9
    out = {
        "metric": ("particle-steps/s, 3-D Ma10 sphere on a body-fitted hexahedral shell" if hexa else
                   "particle-steps/s, 2-D Ma5 cylinder on body-fitted O-grids"),
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64-mixed", "data": "synthetic",
        "config": {"workload": ("Ma 10 argon sphere (R = 1 m, 65 K, wall 302 K) on a 72 x 36 x 76 hexahedral "
                                "shell to 4 R, 400 particles in an outermost equatorial cell, FP32-mixed, "
                                "sampling on") if hexa else
                               ("12 O-grid runs of the Ma 5 argon cylinder (180 nodes around, first layer "
                                "1 mm, growth 1.1 / 1.05, outer radius 3 R, Kn 0.01 / 0.1, 500 particles "
                                "in the outermost cells), FP32-mixed, sampling on"),
                   "particles": int(npart), "cells": ncells},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "move group: k_move_fast (passes mesh waves) + k_move_mesh (face-to-face tracking)",
                     "kernel_ms": r32["tile_ms"], "launches_timed": r32["launches"],
                     "algorithmic_bytes_per_launch": move_bytes},
    }
    if not args.no_fp64:
        del sim32
        import torch
        torch.cuda.empty_cache()
        sim64, r64 = run_gpu("fp64", cases, gas, args.warmup, args.steps, timed_group="move")
        v64 = 0.5 * (r64["n0"] + r64["n1"]) * args.steps / r64["dt"]
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["dt"] / args.steps, "move_ms": r64["tile_ms"]}
        out["mixed_speedup_vs_fp64"] = value / v64
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--develop", type=int, default=2000,
                    help="untimed steps from the impulsive start before the warmup (cylinder), so the "
                         "timed state is the developed flow whatever the warmup")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle steps of the CPU baseline sample")
    ap.add_argument("--workload", choices=("cylinder", "ogrid", "sphere_hex"), default="cylinder")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("ogrid", "sphere_hex"):
        main_ogrid(args)
        return

    import workloads as W
    gas = W.gas()
    case = W.cylinder_2d()
    case["n_steady"] = args.develop + args.warmup      # the timed steps sample (Step 5 is on)
    ncells = case["nx"] * case["ny"]

    log("[bench] fp32-mixed: develop %d, warmup %d, timed %d" % (args.develop, args.warmup, args.steps))
    sim32, r32 = run_gpu("fp32", case, gas, args.warmup, args.steps, develop=args.develop)
    npart = 0.5 * (r32["n0"] + r32["n1"])
    value = npart * args.steps / r32["dt"]
    ms_step = 1e3 * r32["dt"] / args.steps
    tile_bytes = TILE_BYTES_PER_PARTICLE * npart + TILE_BYTES_PER_CELL * ncells
    achieved = tile_bytes / (r32["tile_ms"] * 1e-3) / 1e9
    ratio = committed_traffic_ratio()
    traffic = ratio * tile_bytes if ratio is not None else None
    log("[bench] fp32: %.3f ms/step, %.3e particle-steps/s, tile kernel %.3f ms" % (ms_step, value, r32["tile_ms"]))

    out = {
        "metric": "particle-steps/s, 2-D Ma10 cylinder: FP32-mixed vs FP64 at ≤1e-3 moment error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64-mixed",
        "data": "synthetic",
        "config": {"workload": "2-D Ma10 argon cylinder, Kn 0.01 on D, 800x600 cut-cell grid, 30 particles "
                               "per cell at the freestream density, FP32-mixed, sampling on; timed from %d "
                               "steps after the impulsive start (%s flow: %d particles)"
                               % (r32["before"], "developed" if r32["before"] >= 2000 else "developing",
                                  int(npart)),
                   "particles": int(npart), "cells": ncells,
                   "steps_before_timing": {"develop": args.develop, "warmup": args.warmup,
                                           "autotune": r32["tune"]["steps"]},
                   "launch_grids": {k: v[0] for k, v in r32["tune"]["grids"].items()},
                   "tuning_steps": r32["tune"]["steps"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_collide_tile<float> (NTC, Shakhov, rescale, sampling on LDS tiles)",
                     "kernel_ms": r32["tile_ms"], "launches_timed": r32["launches"],
                     "timing_period": TIMING_PERIOD,
                     "algorithmic_bytes_per_launch": tile_bytes,
                     "valu_active_frac": committed_valu()},
        "step_roofline": step_roofline(value),
    }
    if not args.no_fp64:
        del sim32
        import torch
        torch.cuda.empty_cache()
        log("[bench] fp64: warmup %d, timed %d" % (args.warmup, args.steps))
        sim64, r64 = run_gpu("fp64", case, gas, args.warmup, args.steps, develop=args.develop)
        v64 = 0.5 * (r64["n0"] + r64["n1"]) * args.steps / r64["dt"]
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["dt"] / args.steps, "tile_kernel_ms": r64["tile_ms"]}
        out["mixed_speedup_vs_fp64"] = value / v64
        log("[bench] fp64: %.3f ms/step, %.3e particle-steps/s" % (1e3 * r64["dt"] / args.steps, v64))
        acc = paired_accuracy(sim64, case, gas)
        out["accuracy"] = {"paired_one_step_rel_l2": acc["all_cells"], "bound": 1e-3,
                           "paired_one_step_rel_l2_same_particles": acc["same_particles"],
                           "cells_with_other_particles": acc["cells_with_other_particles"],
                           "occupied_cells": acc["occupied_cells"],
                           "fp64_other_seed_one_step_rel_l2": acc["fp64_other_seed"],
                           "state": "the FP64 run's developed cylinder state after %d steps, imported "
                                    "into an FP32-mixed sim and into an FP64 sim with another seed; one "
                                    "step of each" % (r64["before"] + args.steps),
                           "long_run": "profiles/mixed_accuracy_cylinder_long.md (2000 sampled steps: "
                                       "time averages against the other-seed noise floor, 3-sigma shares)"}
        log("[bench] FP32-mixed vs FP64, one paired step, relative L2: %s" % acc)
        base_sim, base_steps = sim64, r64["before"] + args.steps + 1
    else:
        base_sim, base_steps = sim32, r32["before"] + args.steps
    if not args.no_cpu:
        log("[bench] cpu oracle baseline")
        v_cpu, n_cpu, t_cpu = cpu_baseline(base_sim, case, gas, args.cpu_steps)
        out["cpu_baseline"] = {"value": v_cpu, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": "%d step(s) of the same cylinder workload, single-threaded, from the "
                                         "GPU's FP64 state %d steps after the impulsive start (%d particles, "
                                         "%.1f s)" % (args.cpu_steps, base_steps, n_cpu, t_cpu),
                               "host": host_cpu()}
        log("[bench] cpu: %.3e particle-steps/s (%.1f s)" % (v_cpu, t_cpu))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
