"""Throughput of the PIC cycle on one MI355X: the C1 laser-wakefield workload.

One step = the whole production step of the library (periodic cell sort,
fused cubic gather + Boris push + Esirkepov deposit, current read-out,
perfect-dispersion field update, laser source, window motion and plasma
injection).  The job is the 1000-step C1 run: W warm-up steps, then K timed
steps (defaults 5 + 995).  Prints one JSON line:

  value      particle-steps/s over the timed steps (particles live in HBM
             before timing starts; the count per step is the mean of the
             counts before and after the timed region)
  roofline   the fused tile kernel (dominant): algorithmic bytes per launch
             (60 B per particle read+written, 24 B per cell of E/B read,
             24 B per cell of int64 current accumulated) over its mean
             launch time from HIP events on the library's stream, against
             8 TB/s HBM3E
  cpu_baseline  the FP64 oracle (single thread) on a crop of the same
             workload, gather + push + deposit only
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


def cpu_baseline(cfg, crop=(64, 32, 32), steps=12):
    """Oracle gather+push+deposit rate on a crop of the workload (one thread)."""
    import numpy as np

    from oracle import oracle as O

    g = O.make_grid(crop, cfg["d"], cfg["dt"], solver=cfg["solver"], xbc=1)
    p = cfg["plasma"]
    P = O.make_plasma(p["x_start"], p["ramp"], p["n_plateau"], p["ppc"])
    x, w, _ = O.inject(g, P, 0, 0, crop[0] - 3)
    u = np.zeros_like(x)
    E = O.zeros_field(g)
    B = O.zeros_field(g)
    rng = np.random.default_rng(0)
    E += 0.05 * rng.standard_normal(E.shape)   # a perturbed state so particles move
    t = 0.0
    for _ in range(steps):
        t0 = time.perf_counter()
        x0 = x.copy()
        x, u, x1 = O.push(g, x, u, E, B)
        O.deposit(g, x0, x1, w)
        t += time.perf_counter() - t0
    npart = x.shape[1]
    return {"value": npart * steps / t, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"C1 geometry crop {crop[0]}x{crop[1]}x{crop[2]} cells ({npart} particles, ramp region), "
                      f"{steps} FP64 oracle steps of gather+push+deposit, single thread"}


KERNEL_SOURCES = ("paper_1204_0838_amd/csrc/pic_tile.hip", "paper_1204_0838_amd/csrc/pic_particle_ops.h",
                  "paper_1204_0838_amd/csrc/pic_device.h")


def tile_alg_bytes(npart, ncell, prof):
    """Algorithmic HBM bytes of one tile launch, averaged over the timed
    launches: 60 B per particle (cell, off, u, w read; cell, off, u written)
    and 48 B per cell (E, B staged once; the int64 current added once), plus
    16 B per particle on the launches right after a sort, which do the sort's
    gather (the source index and id read, w and id written)."""
    gather_share = prof["sorts"] / max(1, prof["tile_launches"])
    return (60.0 + 16.0 * gather_share) * npart + 48.0 * ncell


def measured_traffic(path, cfg):
    """HBM bytes per k_pic_tile launch from the committed rocprofv3 counter
    summary, or None when it is missing, for another grid, or the kernel
    sources changed since it was measured."""
    import hashlib

    if cfg["n"] != (512, 256, 256) or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return rec.get("bytes_per_launch") if rec.get("source_sha256") == h.hexdigest() else None


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
    alg_bytes = tile_alg_bytes(npart, ncell, prof)
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
        "gather_push_deposit_particle_steps_per_s": npart * prof["tile_launches"] / (prof["tile_ms"] * 1e-3),
        "phase_ms_per_step": {k[:-3]: prof[k] / max(1, prof["steps"]) for k in
                              ("sort_ms", "tile_ms", "loose_ms", "jpost_ms", "field_ms", "window_ms")},
        "sequential_ms_per_step": seq_ms,
        "batched_speedup_vs_sequential": seq_ms / (ms / K),
        "roofline": {"bound": "hbm", "kernel": "k_batch_tile", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg_bytes, "mean_launch_ms": tile_ms},
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

    cfg = c4._cfg(workloads.C1, c4.PPC2)
    sim = workloads.build(cfg, jpost="denoiser", tuned=False)
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
        "roofline": {"bound": "mfma", "kernel": "denoiser (k_dn_c4, k_dn_c32, k_dn_c3 + output stage)",
                     "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "traffic": None,
                     "alg_flop_per_step": DN_FLOP_PER_CELL * ncell, "mean_denoiser_ms": dn_ms},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=995)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--grid", type=str, default="", help="override nx,ny,nz (default: the C1 grid)")
    ap.add_argument("--tile", type=str, default="")
    ap.add_argument("--sort-interval", type=int, default=0)
    ap.add_argument("--guard", type=int, default=-1)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", type=str, default="", help="per-launch HBM bytes from rocprofv3 counters")
    ap.add_argument("--workload", type=str, default="c1", choices=["c1", "c3", "c4"],
                    help="c1 (default): the LWFA slab; c3: the batched 64-member parameter scan; "
                         "c4: the 2-ppc run with the learned denoiser")
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
        if args.steps == 995:
            args.steps = 195
        bench_c3(args)
        return
    if args.workload == "c4":
        if args.steps == 995:
            args.steps = 200
        bench_c4(args)
        return

    from paper_1204_0838_amd import workloads

    cfg = workloads.C1
    if args.grid:
        cfg = workloads.scaled(cfg, [int(v) for v in args.grid.split(",")])
    tiling = {}
    if args.tile:
        tiling["tile"] = tuple(int(v) for v in args.tile.split(","))
    if args.sort_interval:
        tiling["sort_interval"] = args.sort_interval
    if args.guard >= 0:
        tiling["guard"] = args.guard
    if args.threads:
        tiling["threads"] = args.threads
    t_setup = time.perf_counter()
    sim = workloads.build(cfg, **tiling)
    sim.sync()
    print(f"# setup {time.perf_counter() - t_setup:.1f}s, window starts at step "
          f"{workloads.window_start_step(cfg)}", file=sys.stderr, flush=True)
    done = 0
    while done < args.warmup:
        k = min(100, args.warmup - done)
        sim.step(k)
        done += k
    sim.sync()
    n0 = sim.reduce()["n_particles"]
    sim.profile_enable(True)
    st = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    left = args.steps
    while left > 0:
        k = min(100, left)
        sim.step(k)
        left -= k
        if args.steps >= 200 and left % 200 == 0:
            print(f"# {args.steps - left}/{args.steps} steps", file=sys.stderr, flush=True)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = sim.profile_read()
    n1 = sim.reduce()["n_particles"]
    npart = 0.5 * (n0 + n1)
    K = args.steps
    value = npart * K / (ms * 1e-3)
    ncell = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    launches = max(1, prof["tile_launches"])
    tile_ms = prof["tile_ms"] / launches
    alg_bytes = tile_alg_bytes(npart, ncell, prof)
    achieved = alg_bytes / (tile_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic_json or os.path.join(ROOT, "profiles", "k_pic_tile_C1_traffic.json"),
                               cfg)
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
            "workload": "C1 3D LWFA moving-window slab {}x{}x{}, dx=0.25 dy=dz=0.5 c/wp, perfect-dispersion "
                        "solver c dt = dx, 8 ppc cold lattice plasma behind a 50-cell ramp, a0=4 w0=5 "
                        "FWHM 2.5 laser from the x boundary, window at c, 1000-step run".format(*cfg["n"]),
            "particles": int(npart),
            "cells": ncell,
            "tiling": {"tile": [sim.desc.tile[a] or 8 for a in range(3)],
                       "guard": sim.desc.guard if sim.desc.guard >= 0 else 1,
                       "threads": sim.desc.threads or 512, "interleave": sim.desc.interleave or 8,
                       "sort_interval": sim.desc.sort_interval or 2,
                       "source": "explicit" if tiling else "autotune cache or library default"},
        },
        "gather_push_deposit_particle_steps_per_s": npart * launches / (prof["tile_ms"] * 1e-3),
        "phase_ms_per_step": {k[:-3]: prof[k] / max(1, prof["steps"]) for k in
                              ("sort_ms", "tile_ms", "loose_ms", "jpost_ms", "field_ms", "window_ms")},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_pic_tile",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "mean_launch_ms": tile_ms,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
