"""Fixed workloads for hardware-counter runs (rocprofv3 --pmc), which need a short program.

    python -m paper_2506_23917_amd.profile_workload --warmup 2000 --steps 20
        the bench workload (2-D Ma 10 cylinder, 800 x 600, FP32-mixed): `warmup` steps to
        develop the flow, then `steps` more with sampling on (filter the counters to the
        last launches of the kernel of interest)
    python -m paper_2506_23917_amd.profile_workload --workload jets --warmup 2000 --steps 200
        the ragged batch of 32 planar jets (one launch per kernel for the whole batch, the
        step replayed from a captured graph); `--workload sphere` the 3-D Ma 10 sphere
        (240 x 160 x 160); `--workload sod` 256 replicas of the Sod tube (200 cells, 160 / 20
        particles per cell, graph replay); `--workload relax` the 0-D batch (4096 cells x 1000
        particles from the skewed bi-Maxwellian state); `--workload ogrid` the batch of twelve
        Ma 5 cylinder O-grids; `--workload sphere_hex` the Ma 10 sphere on a hexahedral shell.
        Each prints particle-steps/s of the timed steps (Step 5 sampling on in them); with `--repeats 5` it times five
        windows of `steps` steps one after the other and prints one JSON line with each and
        their median; `--autotune` first picks the launch shapes on the developed flow.
    python -m paper_2506_23917_amd.profile_workload --workload sod --accuracy --warmup 40
        FP32-mixed against FP64 from the same state: the FP64 path runs `warmup` steps, its
        state is imported into an FP32-mixed sim (the first four cases of a batch), both take
        one step with the same random numbers, and the relative L2 differences of the cells'
        n, u, T, q (Eq. 31 estimators of the current particles) are printed
    python -m paper_2506_23917_amd.profile_workload --long-accuracy --warmup 2000 --steps 2000
        the accuracy gate on the cylinder (800 x 600): the flow developed in FP64 for `warmup`
        steps, then from that state `steps` sampled steps each in FP32-mixed (same seed), FP64
        (same seed) and FP64 (another seed), in ten batches; prints one JSON line with the
        relative L2 of the time-averaged n, u, T, q against the same-seed FP64 run (FP32-mixed,
        and the other-seed FP64 run as the noise floor), the share of cells beyond 3 standard
        errors of a difference (from the FP64 run's batch means) and the paired one- and
        ten-step L2 (same imported state and seed)
    python -m paper_2506_23917_amd.profile_workload --dense-census --warmup 2000 --steps 200
        the cylinder's cells above the tile kernel's limit: particles-per-cell histogram after
        `warmup` steps, then the block-per-cell kernels' time (side stream) and the step's, by
        HIP events over `steps` steps after the autotuner
    python -m paper_2506_23917_amd.profile_workload --copy-mib 1024
        a plain device-to-device copy of a known size, to scale the FETCH_SIZE / WRITE_SIZE
        counters to bytes
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--accuracy", action="store_true")
    ap.add_argument("--long-accuracy", action="store_true")
    ap.add_argument("--workload", default="cylinder",
                    choices=["cylinder", "jets", "sphere", "sod", "relax", "ogrid", "sphere_hex"])
    ap.add_argument("--repeats", type=int, default=1,
                    help="time this many windows of --steps steps; print each and their median (one JSON line)")
    ap.add_argument("--autotune", action="store_true", help="pick the launch shapes after the warmup")
    ap.add_argument("--dense-census", action="store_true",
                    help="cylinder: particles-per-cell histogram and the block-per-cell kernel's share and time")
    args = ap.parse_args()
    import torch
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copied %d MiB x 3" % args.copy_mib, flush=True)
        return
    import time
    import workloads as W
    from paper_2506_23917_amd.hs import Sim
    if args.accuracy:
        paired_accuracy(args)
        return
    if args.long_accuracy:
        long_accuracy(args)
        return
    if args.dense_census:
        dense_census(args)
        return
    if args.workload == "jets":
        cases = W.jets_2d()
        for c in cases:
            c["n_steady"] = args.warmup        # the timed steps sample (Step 5 is on)
        sim = Sim(W.gas(), cases, precision=args.precision, device="cuda:0", graph=True)
    elif args.workload == "sod":
        cases = [W.sod_1d(seed=1 + r, n_steady=0) for r in range(256)]
        sim = Sim(W.gas(), cases, precision=args.precision, device="cuda:0", graph=True)
    elif args.workload == "relax":
        import numpy as np
        case = W.relax_0d(n_steady=0)
        cases = [case]
        v, cell, ids = W.relax_0d_state(case)
        sim = Sim(W.gas(), case, precision=args.precision, device="cuda:0", no_particles=True)
        st0 = sim.export_state(0)
        sim.import_state(0, dict(pos=np.zeros((len(ids), 3)), vel=v, cell=cell, id=ids, next_id=len(ids),
                                 step=0, sigc_max=st0["sigc_max"]))
    elif args.workload in ("ogrid", "sphere_hex"):
        cases = W.ogrid_batch() if args.workload == "ogrid" else [W.sphere_hex()]
        for c in cases:
            c["n_steady"] = args.warmup
        sim = Sim(W.gas(), cases, precision=args.precision, device="cuda:0")
    else:
        case = W.cylinder_2d() if args.workload == "cylinder" else W.sphere_3d()
        case["n_steady"] = args.warmup
        cases = [case]
        sim = Sim(W.gas(), case, precision=args.precision, device="cuda:0")
    nc = len(cases)
    done = 0
    while done < args.warmup:
        k = min(500, args.warmup - done)
        sim.step(k)
        sim.sync()
        done += k
        print("warmup %d / %d" % (done, args.warmup), flush=True)
    if args.autotune:
        tune = sim.autotune(steps_per_trial=10)
        print("autotuned: %s (%d steps)" % ({k: v[0] for k, v in tune["grids"].items()}, tune["steps"]), flush=True)
    windows = []
    for rep in range(max(1, args.repeats)):
        n0 = sum(sim.num_particles(c) for c in range(nc))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.steps)
        sim.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n1 = sum(sim.num_particles(c) for c in range(nc))
        windows.append(dict(ms_per_step=1e3 * dt / max(args.steps, 1), particles=0.5 * (n0 + n1),
                            particle_steps_per_s=0.5 * (n0 + n1) * args.steps / dt))
        print("timed steps %d, particles %d, %.4f ms/step, %.4e particle-steps/s" %
              (args.steps, n1, windows[-1]["ms_per_step"], windows[-1]["particle_steps_per_s"]), flush=True)
    if args.repeats > 1:
        import json
        import statistics
        med = statistics.median(w["particle_steps_per_s"] for w in windows)
        print(json.dumps(dict(workload=args.workload, precision=args.precision, warmup=args.warmup, steps=args.steps,
                              repeats=args.repeats, median_particle_steps_per_s=med,
                              median_ms_per_step=statistics.median(w["ms_per_step"] for w in windows),
                              particles=statistics.median(w["particles"] for w in windows), windows=windows)),
              flush=True)


def dense_census(args):
    """The developed cylinder after `warmup` steps: histogram of particles per cell, the cells
    above the tile kernel's limit (192) and their particles, then `steps` steps with the launch
    shapes the autotuner picks and HIP events around the block-per-cell kernels (on the side
    stream) and around the whole step; one JSON line."""
    import json
    import numpy as np
    import workloads as W
    from paper_2506_23917_amd.hs import Sim
    case = W.cylinder_2d()
    case["n_steady"] = args.warmup
    sim = Sim(W.gas(), case, precision=args.precision, device="cuda:0")
    done = 0
    while done < args.warmup:
        k = min(500, args.warmup - done)
        sim.step(k)
        sim.sync()
        done += k
    st = sim.export_state(0)
    cnt = np.bincount(st["cell"], minlength=case["nx"] * case["ny"])
    edges = [(0, 0), (1, 9), (10, 19), (20, 39), (40, 63), (64, 127), (128, 192), (193, 512), (513, 1024),
             (1025, 2048), (2049, 4096), (4097, 1 << 30)]
    hist = [dict(lo=a, hi=b, cells=int(((cnt >= a) & (cnt <= b)).sum()), particles=int(cnt[(cnt >= a) & (cnt <= b)].sum()))
            for a, b in edges]
    dense = cnt > 192
    tune = sim.autotune(steps_per_trial=10)
    sim.set_timing(["dense", "step"])
    sim.clear_timing()
    sim.step(args.steps)
    sim.sync()
    print(json.dumps(dict(workload="cylinder", precision=args.precision, step=int(st["step"]), particles=int(cnt.sum()),
                          cells=int(cnt.size), dense_cells=int(dense.sum()), dense_particles=int(cnt[dense].sum()),
                          densest=int(cnt.max()), histogram=hist, launch_grids={k: v[0] for k, v in tune["grids"].items()},
                          timed_steps=args.steps, dense_ms=sim.kernel_timing("dense")[0],
                          step_ms=sim.kernel_timing("step")[0])), flush=True)


def _cases(name, warmup):
    import workloads as W
    if name == "cylinder":
        return [W.cylinder_2d()]
    if name == "sphere":
        return [W.sphere_3d()]
    if name == "jets":
        return W.jets_2d()[:4]
    if name == "sod":
        return [W.sod_1d(seed=1 + r) for r in range(4)]
    if name == "relax":
        return [W.relax_0d()]
    return W.ogrid_batch()[:4]


def paired_accuracy(args):
    import numpy as np
    import workloads as W
    from paper_2506_23917_amd.hs import Sim
    gas = W.gas()
    cases = _cases(args.workload, args.warmup)
    if args.workload == "relax":
        s64 = Sim(gas, cases, precision="fp64", device="cuda:0", no_particles=True)
        v, cell, ids = W.relax_0d_state(cases[0])
        st0 = s64.export_state(0)
        s64.import_state(0, dict(pos=np.zeros((len(ids), 3)), vel=v, cell=cell, id=ids, next_id=len(ids),
                                 step=0, sigc_max=st0["sigc_max"]))
    else:
        s64 = Sim(gas, cases, precision="fp64", device="cuda:0")
    done = 0
    while done < args.warmup:
        k = min(500, args.warmup - done)
        s64.step(k)
        s64.sync()
        done += k
    s32 = Sim(gas, cases, precision="fp32", device="cuda:0", no_particles=True)
    for c in range(len(cases)):
        s32.import_state(c, s64.export_state(c))
    s64.step(1)
    s32.step(1)
    a = [s32.sample_moments(c, mode=1) for c in range(len(cases))]
    b = [s64.sample_moments(c, mode=1) for c in range(len(cases))]
    cat = lambda L, k: np.concatenate([np.asarray(x[k]).reshape(len(x["n"]), -1) for x in L])
    n32, n64 = cat(a, "n"), cat(b, "n")
    sel = (n64[:, 0] > 0)
    rel = lambda x, y: float(np.sqrt(np.sum((x - y) ** 2)) / max(np.sqrt(np.sum(y ** 2)), 1e-300))
    out = {k: rel(cat(a, k)[sel], cat(b, k)[sel]) for k in ("n", "T", "q")}
    u32, u64, T64 = cat(a, "u")[sel], cat(b, "u")[sel], cat(b, "T")[sel]
    scale = np.sqrt(np.sum(u64 ** 2) + np.sum(1.380649e-23 * np.maximum(T64, 0.0) / gas["m"]))
    out["u"] = float(np.sqrt(np.sum((u32 - u64) ** 2)) / scale)
    print("accuracy %s cases %d cells %d after %d FP64 steps: n %.3e u %.3e T %.3e q %.3e" %
          (args.workload, len(cases), int(sel.sum()), args.warmup, out["n"], out["u"], out["T"], out["q"]), flush=True)


def _acc_moments(acc, steps, m=6.63e-26, kb=1.380649e-23):
    """Step (6) averages over `steps` sampled steps from 13-sum arrays (cells, 13): n (up to
    the factor F_N / V), u (3), T, q (3, up to the same factor); zero where a cell has no
    samples."""
    import numpy as np
    N = acc[:, 0]
    ok = N > 0
    Ns = np.where(ok, N, 1.0)
    U = acc[:, 1:4] / Ns[:, None]
    cc = (acc[:, 4] + acc[:, 5] + acc[:, 6]) / Ns
    uu = (U ** 2).sum(1)
    cij = np.stack([np.stack([acc[:, 4], acc[:, 7], acc[:, 8]], 1),
                    np.stack([acc[:, 7], acc[:, 5], acc[:, 9]], 1),
                    np.stack([acc[:, 8], acc[:, 9], acc[:, 6]], 1)], 1) / Ns[:, None, None]
    uc = np.einsum("kab,kb->ka", cij, U)
    n = N / steps
    q = 0.5 * m * n[:, None] * (acc[:, 10:13] / Ns[:, None] - 2 * uc - U * cc[:, None] + 2 * U * uu[:, None])
    T = m / (3 * kb) * (cc - uu)
    z = lambda x: np.where(ok if x.ndim == 1 else ok[:, None], x, 0.0)
    return dict(n=n, u=z(U), T=z(T), q=z(q))


def long_accuracy(args):
    import json
    import numpy as np
    import workloads as W
    from paper_2506_23917_amd.hs import Sim
    gas = W.gas()
    case = W.cylinder_2d()
    s64 = Sim(gas, case, precision="fp64", device="cuda:0")
    done = 0
    while done < args.warmup:
        k = min(500, args.warmup - done)
        s64.step(k)
        s64.sync()
        done += k
        print("fp64 development %d / %d" % (done, args.warmup), flush=True)
    st0 = s64.export_state(0)
    del s64
    rel = lambda x, y: float(np.sqrt(np.sum((x - y) ** 2)) / max(np.sqrt(np.sum(y ** 2)), 1e-300))

    def l2(a, b, sel):
        out = {k: rel(np.asarray(a[k])[sel], np.asarray(b[k])[sel]) for k in ("n", "T", "q")}
        u_a, u_b, T_b = np.asarray(a["u"]).reshape(-1, 3)[sel], np.asarray(b["u"]).reshape(-1, 3)[sel], np.asarray(b["T"])[sel]
        scale = np.sqrt(np.sum(u_b ** 2) + np.sum(1.380649e-23 * np.maximum(T_b, 0.0) / gas["m"]))
        out["u"] = float(np.sqrt(np.sum((u_a - u_b) ** 2)) / scale)
        return out

    # paired short horizons: one and ten steps from the same state and seed; beside them, an
    # FP64 run with another seed from the same state (the noise of the current-state moments)
    paired, paired_noise = {}, {}
    p32 = Sim(gas, case, precision="fp32", device="cuda:0", no_particles=True)
    p64 = Sim(gas, case, precision="fp64", device="cuda:0", no_particles=True)
    p64b = Sim(gas, dict(case, seed=977), precision="fp64", device="cuda:0", no_particles=True)
    for sim in (p32, p64, p64b):
        sim.import_state(0, st0)
    for k, nsteps in (("1", 1), ("10", 9)):
        for sim in (p32, p64, p64b):
            sim.step(nsteps)
        a, b, c = p32.sample_moments(0, mode=1), p64.sample_moments(0, mode=1), p64b.sample_moments(0, mode=1)
        paired[k] = l2(a, b, np.asarray(b["n"]) > 0)
        paired_noise[k] = l2(c, b, np.asarray(b["n"]) > 0)
    del p32, p64, p64b
    print("paired", paired, "noise", paired_noise, flush=True)

    nb = 10
    per = max(1, args.steps // nb)
    runs = {}
    for name, prec, seed in (("fp32", "fp32", case["seed"]), ("fp64", "fp64", case["seed"]), ("fp64b", "fp64", 977)):
        c = dict(case, seed=seed, n_steady=args.warmup)
        sim = Sim(gas, c, precision=prec, device="cuda:0", no_particles=True)
        sim.import_state(0, st0)
        prev = None
        batches = []
        for b in range(nb):
            sim.step(per)
            acc = sim.export_state(0)["acc"].copy()
            batches.append(acc - (prev if prev is not None else 0.0))
            prev = acc
        runs[name] = dict(final=sim.sample_moments(0, mode=0), acc=prev, batches=batches)
        print("%s: %d sampled steps" % (name, runs[name]["final"]["n_samples"]), flush=True)
        del sim
    sel_all = np.asarray(runs["fp64"]["final"]["n"]) > 0
    long_l2 = {"fp32_mixed_vs_fp64": l2(runs["fp32"]["final"], runs["fp64"]["final"], sel_all),
               "fp64_other_seed_vs_fp64": l2(runs["fp64b"]["final"], runs["fp64"]["final"], sel_all)}
    # 3-sigma: z of each cell's average against the same-seed FP64 run, in standard errors of a
    # difference of two independent runs (batch means of the FP64 run); cells with at least 20
    # particles in every batch
    bm = [_acc_moments(b, per) for b in runs["fp64"]["batches"]]
    nmin = np.min([b[:, 0] for b in runs["fp64"]["batches"]], axis=0)
    base = nmin >= 20 * per
    pooled = {k: _acc_moments(runs[k]["acc"], nb * per) for k in runs}
    sigma = {}
    for k in ("n", "u", "T", "q"):
        arr = np.array([x[k] for x in bm])
        se = arr.std(0, ddof=1) / np.sqrt(nb) * np.sqrt(2)
        sel = (base if se.ndim == 1 else base[:, None]) & (se > 0)
        res = {}
        for other in ("fp32", "fp64b"):
            z = (pooled[other][k][sel] - pooled["fp64"][k][sel]) / se[sel]
            res[other] = {"beyond_3sigma": float((np.abs(z) > 3).mean()), "mean_z2": float((z ** 2).mean()),
                          "values": int(z.size)}
        sigma[k] = res
    out = {"workload": "2-D Ma10 argon cylinder 800x600, developed %d FP64 steps, then %d sampled steps per run"
                       % (args.warmup, nb * per),
           "cells_compared": int(sel_all.sum()), "cells_in_3sigma_test": int(base.sum()),
           "paired_l2": paired, "paired_l2_fp64_other_seed": paired_noise, "time_average_l2": long_l2,
           "three_sigma": sigma,
           "z_reference": "Student t, 9 degrees of freedom: mean z^2 = 9/7 = 1.29, P(|z| > 3) = 0.015"}
    print("LONG_ACCURACY " + json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
