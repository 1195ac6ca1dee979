"""Throughput of the PIC cycle on one MI355X: the C1 laser-wakefield workload.

One step = the whole production step of the library (periodic cell sort,
fused cubic gather + Boris push + Esirkepov deposit, current read-out,
perfect-dispersion field update, laser source, window motion and plasma
injection).  The job is the 1000-step C1 run.  Its cost changes over the run
(early on the laser has not reached the plasma and the cold particles do
not move, so they deposit nothing; later the wake makes most of them move),
so the K timed steps are spread evenly over the run: after W untimed
warm-up steps, step W + floor((j + 1/2)(1000 - W)/K) is timed for j < K and
the steps between are advanced untimed.  K = 1000 - W times every step.
Each timed step is bracketed by device synchronisations and HIP events on
the library's stream.  Prints one JSON line:

  value      particle-steps/s over the timed steps (particles live in HBM;
             the count of each timed step is the live count before it)
  roofline   the fused tile kernel (dominant): algorithmic bytes per launch
             (60 B per particle read+written, 24 B per cell of E/B read,
             24 B per cell of int64 current accumulated) over its mean
             launch time from HIP events on the library's stream, against
             8 TB/s HBM3E; the sort's gather, which the launch after a sort
             also does, is reported apart
  cpu_baseline  the FP64 oracle (single thread) on a crop of the same
             workload, gather + push + deposit only, and on the 16-step C0
             parity workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _host_cpu():
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
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail}


def _oracle_gpd(O, g, x, u, w, E, B, steps, field_steps=False):
    """Time `steps` oracle gather+push+deposit passes (the field update, when
    run, is untimed); returns (seconds, particle-steps)."""
    t = 0.0
    ps = 0
    for _ in range(steps):
        t0 = time.perf_counter()
        x0 = x.copy()
        x, u, x1 = O.push(g, x, u, E, B)
        J = O.deposit(g, x0, x1, w)
        t += time.perf_counter() - t0
        ps += x.shape[1]
        if field_steps:
            E, B = O.field_step(g, E, B, J)
    return t, ps


def cpu_baseline(cfg, crop=(64, 32, 32), steps=12):
    """Oracle gather+push+deposit rate on a crop of the workload (one thread),
    and on the 16-step C0 parity workload."""
    import numpy as np

    from oracle import oracle as O
    from paper_1204_0838_amd import inputs

    g = O.make_grid(crop, cfg["d"], cfg["dt"], solver=cfg["solver"], xbc=1)
    p = cfg["plasma"]
    P = O.make_plasma(p["x_start"], p["ramp"], p["n_plateau"], p["ppc"])
    x, w, _ = O.inject(g, P, 0, 0, crop[0] - 3)
    u = np.zeros_like(x)
    E = O.zeros_field(g)
    B = O.zeros_field(g)
    rng = np.random.default_rng(0)
    E += 0.05 * rng.standard_normal(E.shape)   # a perturbed state so particles move and deposit
    t, ps = _oracle_gpd(O, g, x, u, w, E, B, steps)
    npart = x.shape[1]
    # C0: 64x32x32 periodic Yee grid, 524,288 electrons, 16 full steps (field update untimed)
    c0g = inputs.c0_grid()
    pl = inputs.c0_particles(seed=1)
    og = O.from_grid(c0g)
    t0, ps0 = _oracle_gpd(O, og, pl.positions(c0g), pl.u.astype(np.float64), pl.w.astype(np.float64),
                          O.zeros_field(og), O.zeros_field(og), 16, field_steps=True)
    return {"value": ps / t, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"C1 geometry crop {crop[0]}x{crop[1]}x{crop[2]} cells ({npart} particles, ramp region, "
                      f"perturbed E so that particles move), {steps} FP64 oracle steps of gather+push+deposit, "
                      f"single thread",
            "host": _host_cpu(),
            "c0_16_steps": {"value": ps0 / t0, "unit": "particle-steps/s", "cores": 1,
                            "sample": "C0 64x32x32 periodic Yee grid, 524,288 electrons, 16 FP64 oracle steps, "
                                      "gather+push+deposit timed (field update untimed), single thread"}}


KERNEL_SOURCES = ("paper_1204_0838_amd/csrc/pic_tile.hip", "paper_1204_0838_amd/csrc/pic_particle_ops.h",
                  "paper_1204_0838_amd/csrc/pic_device.h")


def tile_alg_bytes(npart, ncell):
    """Algorithmic HBM bytes of one tile launch: 60 B per particle (cell, off,
    u, w read; cell, off, u written) and 48 B per cell (E, B staged once; the
    int64 current added once)."""
    return 60.0 * npart + 48.0 * ncell


def sort_gather_bytes(npart, prof):
    """Per tile launch, averaged over the timed launches: the sort's gather
    that the launch right after a sort does (source index and id read, w and
    id written: 16 B per particle) -- sort traffic, not gather+push+deposit."""
    return 16.0 * npart * prof["sorts"] / max(1, prof["tile_launches"])


def measured_traffic(path, cfg, idx):
    """HBM bytes per k_pic_tile launch from the committed rocprofv3 counter
    summary, averaged over the timed steps `idx` (the summary holds the bytes
    of each launch of the run: one launch per step), or None when it is
    missing, for another grid, or the kernel sources changed since it was
    measured."""
    import hashlib

    if cfg["n"] != (512, 256, 256) or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    per_step = rec.get("mb_per_launch_by_step")
    if rec.get("source_sha256") != h.hexdigest() or not per_step or max(idx) >= len(per_step):
        return None
    return 1e6 * sum(per_step[i] for i in idx) / len(idx)


def bench_c3(args):
    """C3: the 64-member parameter scan advanced by the batched launcher
    (one launch per phase for all members), W warm-up + K timed batch steps
    (defaults 5 + 195 of the 200-step scan); then the same members advanced
    one after another with pic_step for a few steps, for comparison."""
    import torch

    from paper_1204_0838_amd import autotune, workloads

    cfgs = workloads.c3_members()
    tilings = [autotune.load_class(workloads.size_class(c), c) or {} for c in cfgs]
    t_setup = time.perf_counter()
    sims, batch = workloads.build_batch(cfgs, tilings=tilings)
    batch.sync()
    print(f"# setup {time.perf_counter() - t_setup:.1f}s, {len(sims)} members", file=sys.stderr, flush=True)
    batch.step(args.warmup)
    batch.sync()

    def live():
        return sum(s.reduce()["n_particles"] for s in sims)

    n0 = live()
    batch.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(batch.stream)
    left = args.steps
    while left > 0:
        k = min(50, left)
        batch.step(k)
        left -= k
        print(f"# {args.steps - left}/{args.steps} batch steps", file=sys.stderr, flush=True)
    e1.record(batch.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = batch.profile_read()
    batch.sync()
    n1 = live()
    npart = 0.5 * (n0 + n1)
    K = args.steps
    ncell = sum(c["n"][0] * c["n"][1] * c["n"][2] for c in cfgs)
    tile_ms = prof["tile_ms"] / max(1, prof["tile_launches"])
    alg_bytes = tile_alg_bytes(npart, ncell)
    achieved = alg_bytes / (tile_ms * 1e-3) / 1e9
    # the same members one after another (per-member launches), a few steps
    seq_steps = 10
    torch.cuda.synchronize()
    e0.record(batch.stream)
    for s in sims:
        s.step(seq_steps)
    e1.record(batch.stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1) / seq_steps
    out = {
        "metric": "particle-steps/s (gather+push+deposit), batched parameter scan",
        "value": npart * K / (ms * 1e-3),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C3 parameter scan: 64 LWFA instances (nx 64..256, ny, nz 32..64, a0 2..5, "
                               "plateau density 0.5..2, 8 ppc, C1 spacings/solver/laser), 200 steps, one launch "
                               "per phase for all members",
                   "members": len(sims), "particles": int(npart), "cells": ncell,
                   "tiling_by_class": {k: v for k, v in zip([workloads.size_class(c) for c in cfgs], tilings)}},
        "gather_push_deposit_particle_steps_per_s": npart * prof["steps"] / ((prof["tile_ms"] + prof["loose_ms"])
                                                                             * 1e-3),
        "phase_ms_per_step": {k[:-3]: prof[k] / max(1, prof["steps"]) for k in
                              ("sort_ms", "tile_ms", "loose_ms", "jpost_ms", "field_ms", "window_ms")},
        "sequential_ms_per_step": seq_ms,
        "batched_speedup_vs_sequential": seq_ms / (ms / K),
        "roofline": {"bound": "hbm", "kernel": "k_batch_tile", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg_bytes, "sort_gather_bytes_per_launch": sort_gather_bytes(npart, prof),
                     "mean_launch_ms": tile_ms},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


DN_FLOP_PER_CELL = 2 * (27 * 3) * 32 + 2 * (27 * 32) * 32 + 2 * (27 * 32) * 3   # three conv layers (65,664)
BF16_MFMA_PEAK_TFLOPS = 2500.0


def bench_c4(args):
    """C4: the C1 geometry at 2 ppc with the learned current denoiser in every
    step (W warm-up + K timed steps).  The roofline line is the denoiser's:
    algorithmic conv flops per step over its measured time, against the dense
    bf16 matrix-core peak.  Weights: the binomial start (zero last layer) with
    random first layers -- the matrix-core work does not depend on the values."""
    import numpy as np
    import torch

    from paper_1204_0838_amd import c4, workloads

    cfg = c4.c4_config()
    sim = workloads.build(cfg, jpost="denoiser")   # (the autotuner's tiling for it when cached)
    sim.set_denoiser(c4.binomial_init(np.random.default_rng(0)), [0.01, 0.01, 0.01])
    sim.step(args.warmup)
    sim.sync()
    n0 = sim.reduce()["n_particles"]
    sim.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    left = args.steps
    while left > 0:
        k = min(100, left)
        sim.step(k)
        left -= k
        print(f"# {args.steps - left}/{args.steps} steps", file=sys.stderr, flush=True)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = sim.profile_read()
    n1 = sim.reduce()["n_particles"]
    npart = 0.5 * (n0 + n1)
    ncell = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    K = args.steps
    dn_ms = prof["jpost_ms"] / max(1, prof["steps"])
    achieved = DN_FLOP_PER_CELL * ncell / (dn_ms * 1e-3) / 1e12
    out = {
        "metric": "steps/s of the 2-ppc denoised run (C4), denoiser matrix-core throughput",
        "value": npart * K / (ms * 1e-3),
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 conv / f32 PIC", "data": "synthetic",
        "config": {"workload": "C4: C1 geometry 512x256x256 at 2 ppc (1x1x2 lattice) with the learned current "
                               "denoiser (3x3x3 conv 3-32-32-3, bf16 MFMA) in every step",
                   "particles": int(npart), "cells": ncell},
        "phase_ms_per_step": {k[:-3]: prof[k] / max(1, prof["steps"]) for k in
                              ("sort_ms", "tile_ms", "loose_ms", "jpost_ms", "field_ms", "window_ms")},
        "roofline": {"bound": "mfma", "kernel": "denoiser (k_dn_c4, k_dn_conv32<0>, k_dn_conv32<2>, k_dn_output)",
                     "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "traffic": None,
                     "alg_flop_per_step": DN_FLOP_PER_CELL * ncell, "mean_denoiser_ms": dn_ms},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


CIRC_CELL_BYTES = 18 * 4 + 9 * 8     # mode-field planes staged once, int64 current channels added once


def cpu_baseline_c2(cfg, crop=(256, 64), steps=20):
    """Cylindrical oracle gather+push+deposit on a crop of the C2 grid (one
    thread): the C2 plasma over a 256x64 (z, r) crop, perturbed fields."""
    import numpy as np

    from oracle import circ as OC
    from paper_1204_0838_amd import inputs

    nz, nr = crop
    g = OC.make_grid(nz, nr, cfg["dz"], cfg["dr"], cfg["dt"])
    p = dict(cfg["plasma"])
    P = OC.load(g, {k: p[k] for k in ("z_start", "ramp", "n_plateau", "ppc")}, 0, 0, nz - 2,
                lambda c: inputs.uniform53(p["seed"], c), nr - 4)
    x, w = P["x"], P["w"].astype(np.float64)
    u = np.zeros_like(x)
    rng = np.random.default_rng(0)
    E = OC.zeros_field(g) + 0.05 * rng.standard_normal((2, 3, nr, nz))
    B = OC.zeros_field(g)
    t = 0.0
    for _ in range(steps):
        t0 = time.perf_counter()
        u, x1 = OC.push(g, x, u, E, B)
        OC.deposit(g, x, x1, u, w)
        t += time.perf_counter() - t0
        x = x1
    return {"value": x.shape[1] * steps / t, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"C2 geometry crop {nz}x{nr} (z, r) cells ({x.shape[1]} particles, 32 per cell, ramp region), "
                      f"{steps} FP64 oracle steps of gather+push+deposit, single thread", "host": _host_cpu()}


def bench_c2(args):
    """C2: the quasi-cylindrical two-mode run, K timed steps spread over its
    2000 steps (as for C1).  Roofline of the fused tile kernel: 60 B per
    particle plus 144 B per (z, r) cell (18 mode-field planes read, 9 int64
    current channels accumulated)."""
    import torch

    from paper_1204_0838_amd import workloads

    cfg = workloads.C2
    total = cfg["steps"]
    args.steps = args.steps or total - args.warmup
    t_setup = time.perf_counter()
    sim = workloads.build_c2(cfg, sort_interval=args.sort_interval, interleave=max(0, args.interleave),
                             threads=args.threads)
    sim.sync()
    idx = timed_indices(total, args.warmup, args.steps, sim.desc.sort_interval or 2)
    print(f"# setup {time.perf_counter() - t_setup:.1f}s, window from step {workloads.c2_window_start(cfg)}, "
          f"{len(idx)} timed steps from {idx[0]} to {idx[-1]}", file=sys.stderr, flush=True)
    st = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    keys = ("sort_ms", "tile_ms", "loose_ms", "jpost_ms", "field_ms", "window_ms", "steps", "sorts", "tile_launches")
    prof = {k: 0 for k in keys}
    ms = part = 0.0
    done = 0
    last = time.perf_counter()
    for j, i in enumerate(idx):
        while done < i:
            k = min(20, i - done)
            sim.step(k)
            done += k
            sim.sync()                        # (progress lines follow the device, also under a profiler)
            if time.perf_counter() - last > 20:
                print(f"# advanced to step {done}", file=sys.stderr, flush=True)
                last = time.perf_counter()
        sim.sync()
        n_live = sim.reduce()["n_particles"]
        sim.profile_enable(True)
        torch.cuda.synchronize()
        e0.record(st)
        sim.step(1)
        e1.record(st)
        torch.cuda.synchronize()
        done += 1
        ms += e0.elapsed_time(e1)
        p = sim.profile_read()
        sim.profile_enable(False)
        for k in keys:
            prof[k] += p[k]
        part += n_live
        if time.perf_counter() - last > 20 or j + 1 == len(idx):
            print(f"# {j + 1}/{len(idx)} timed steps (step {i})", file=sys.stderr, flush=True)
            last = time.perf_counter()
    K = len(idx)
    npart = part / K
    ncell = cfg["nz"] * cfg["nr"]
    launches = max(1, prof["tile_launches"])
    tile_ms = prof["tile_ms"] / launches
    alg = 60.0 * npart + CIRC_CELL_BYTES * ncell
    achieved = alg / (tile_ms * 1e-3) / 1e9
    out = {
        "metric": "particle-steps/s (gather+push+deposit), quasi-cylindrical m=0,1",
        "value": part / (ms * 1e-3), "unit": "particle-steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2 quasi-cylindrical two-mode run Nz=4096 Nr=256 dz=0.05 dr=0.2 c/wp, 32 ppc per "
                               "(z,r) cell at random azimuth, C1 laser on mode 1 and C1 density profile, c dt = dz/2, "
                               "window from step {}, {}-step run; {} timed steps spread over steps {}-{}".format(
                                   workloads.c2_window_start(cfg), total, K, idx[0], idx[-1]),
                   "timed_step_indices": idx if K <= 50 else "{}..{}".format(idx[0], idx[-1]),
                   "particles": int(npart), "cells": ncell, "tile": [32, 8], "guard": 1,
                   "sort_interval": sim.desc.sort_interval or 2, "interleave": sim.desc.interleave or 32,
                   "threads": sim.desc.threads or 512},
        "gather_push_deposit_particle_steps_per_s": part / ((prof["tile_ms"] + prof["loose_ms"]) * 1e-3),
        "phase_ms_per_step": {k[:-3]: prof[k] / max(1, prof["steps"]) for k in keys[:6]},
        "roofline": {"bound": "hbm", "kernel": "k_circ_tile", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None, "alg_bytes_per_launch": alg,
                     "mean_launch_ms": tile_ms},
        "cpu_baseline": None,
    }
    sim.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_c2(cfg)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default: every step after the warm-up)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--grid", type=str, default="", help="override nx,ny,nz (default: the C1 grid)")
    ap.add_argument("--tile", type=str, default="")
    ap.add_argument("--sort-interval", type=int, default=0)
    ap.add_argument("--guard", type=int, default=-1)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--interleave", type=int, default=-1,
                    help="in-tile order of the sort: 0 level order, D >= 1 the transpose depth (default: tuned / library)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", type=str, default="", help="per-launch HBM bytes from rocprofv3 counters")
    ap.add_argument("--workload", type=str, default="c1", choices=["c1", "c1p", "c2", "c3", "c4"],
                    help="c1 (default): the LWFA slab; c1p: the same inside a 16-cell transverse PML; c2: the "
                         "quasi-cylindrical two-mode run; c3: the batched 64-member parameter scan; c4: the 2-ppc "
                         "run with the learned denoiser")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 1 GiB (reference for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "copies": 5}))
        return

    if args.workload == "c3":
        args.steps = args.steps or 195
        bench_c3(args)
        return
    if args.workload == "c4":
        args.steps = args.steps or 200
        bench_c4(args)
        return
    if args.workload == "c2":
        bench_c2(args)
        return
    args.steps = args.steps or 1000 - args.warmup

    bench_c1(args)


def timed_indices(total, warmup, k, period=1):
    """K step indices spread evenly over [warmup, total) (all of them when k =
    total - warmup): the j-th lies in the j-th of k equal, disjoint stretches.
    The cell sort runs on the steps whose index is a multiple of `period`
    (the sort interval); where a stretch holds at least `period` steps, its
    index is the one of residue j mod period nearest the stretch's middle, so
    the timed steps include sorting steps in the run's own proportion (exactly
    when period divides k)."""
    span = total - warmup
    if k >= span:
        return list(range(warmup, total))
    out = []
    for j in range(k):
        lo = warmup + (j * span) // k
        hi = warmup + ((j + 1) * span) // k          # exclusive; hi > lo since span > k
        mid = (lo + hi - 1) // 2
        i = mid
        if period > 1 and hi - lo >= period:
            want = j % period
            cands = [v for v in range(lo, hi) if v % period == want]
            i = min(cands, key=lambda v: abs(v - mid))
        out.append(i)
    return out


def bench_c1(args):
    import torch

    from paper_1204_0838_amd import workloads

    cfg = workloads.C1P if args.workload == "c1p" else workloads.C1
    if args.grid:
        cfg = workloads.scaled(cfg, [int(v) for v in args.grid.split(",")])
    total = cfg["steps"]
    if args.warmup + args.steps > total:
        print(f"warmup + steps must not exceed the {total}-step run", file=sys.stderr)
        sys.exit(2)
    tiling = {}
    if args.tile:
        tiling["tile"] = tuple(int(v) for v in args.tile.split(","))
    if args.sort_interval:
        tiling["sort_interval"] = args.sort_interval
    if args.guard >= 0:
        tiling["guard"] = args.guard
    if args.threads:
        tiling["threads"] = args.threads
    if args.interleave >= 0:
        tiling["interleave"] = args.interleave
    t_setup = time.perf_counter()
    sim = workloads.build(cfg, **tiling)
    sim.sync()
    idx = timed_indices(total, args.warmup, args.steps, sim.desc.sort_interval or 2)
    print(f"# setup {time.perf_counter() - t_setup:.1f}s, window starts at step "
          f"{workloads.window_start_step(cfg)}, {len(idx)} timed steps from {idx[0]} to {idx[-1]}",
          file=sys.stderr, flush=True)
    st = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    keys = ("sort_ms", "tile_ms", "loose_ms", "jpost_ms", "field_ms", "window_ms", "steps", "sorts", "tile_launches")
    prof = {k: 0 for k in keys}
    ms = 0.0
    part_steps = 0.0
    part_launches = 0.0
    done = 0
    last_note = time.perf_counter()
    for j, i in enumerate(idx):
        while done < i:                       # untimed advance to the next timed step
            k = min(10, i - done)
            sim.step(k)
            done += k
            sim.sync()                        # (progress lines follow the device, also under a profiler)
            if time.perf_counter() - last_note > 20:
                print(f"# advanced to step {done}", file=sys.stderr, flush=True)
                last_note = time.perf_counter()
        sim.sync()
        n_live = sim.reduce()["n_particles"]
        sim.profile_enable(True)
        torch.cuda.synchronize()
        e0.record(st)
        sim.step(1)
        e1.record(st)
        torch.cuda.synchronize()
        done += 1
        ms += e0.elapsed_time(e1)
        p = sim.profile_read()
        sim.profile_enable(False)
        for k in keys:
            prof[k] += p[k]
        part_steps += n_live
        part_launches += n_live * p["tile_launches"]
        if time.perf_counter() - last_note > 20 or j + 1 == len(idx):
            print(f"# {j + 1}/{len(idx)} timed steps (step {i})", file=sys.stderr, flush=True)
            last_note = time.perf_counter()
    K = len(idx)
    value = part_steps / (ms * 1e-3)
    npart = part_steps / K                    # mean live particles over the timed steps
    ncell = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    launches = max(1, prof["tile_launches"])
    tile_ms = prof["tile_ms"] / launches
    alg_bytes = tile_alg_bytes(part_launches / launches, ncell)
    achieved = alg_bytes / (tile_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic_json or os.path.join(ROOT, "profiles", "k_pic_tile_C1_traffic.json"),
                               cfg, idx)
    out = {
        "metric": "particle-steps/s (gather+push+deposit), % HBM peak; plain vs denoised at eps",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "{} 3D LWFA moving-window slab {}x{}x{}{}, dx=0.25 dy=dz=0.5 c/wp, perfect-dispersion "
                        "solver c dt = dx, 8 ppc cold lattice plasma behind a 50-cell ramp, a0=4 w0=5 "
                        "FWHM 2.5 laser from the x boundary, window at c from step {}, {}-step run; timed steps "
                        "{}: {} spread evenly over steps {}-{} (untimed advance between them)".format(
                            cfg["name"], *cfg["n"],
                            " with a {}-cell transverse PML".format(cfg["pml"]) if cfg.get("pml") else "",
                            workloads.window_start_step(cfg), total, K,
                            "every step" if K == total - args.warmup else "one in ~{}".format(
                                round((total - args.warmup) / K)), idx[0], idx[-1]),
            "timed_step_indices": idx if K <= 50 else "{}..{}".format(idx[0], idx[-1]),
            "particles": int(npart),
            "cells": ncell,
            "tiling": {"tile": [sim.desc.tile[a] or 8 for a in range(3)],
                       "guard": sim.desc.guard if sim.desc.guard >= 0 else 1,
                       "threads": sim.desc.threads or 512, "interleave": sim.desc.interleave,
                       "sort_interval": sim.desc.sort_interval or 2,
                       "source": "explicit" if tiling else "autotune cache or library default"},
        },
        "gather_push_deposit_particle_steps_per_s": part_steps / ((prof["tile_ms"] + prof["loose_ms"]) * 1e-3),
        "phase_ms_per_step": {k[:-3]: prof[k] / max(1, prof["steps"]) for k in keys[:6]},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_pic_tile",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "sort_gather_bytes_per_launch": sort_gather_bytes(npart, prof),
            "mean_launch_ms": tile_ms,
        },
        "cpu_baseline": None,
    }
    sim.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
