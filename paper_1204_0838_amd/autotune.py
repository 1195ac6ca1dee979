"""Autotuner of the fused step's tiling: tile shape, drift guard, threads per
workgroup, in-tile interleave depth and sort interval.

It times ``pic_step`` on a live simulation for each candidate, switching the
tiling with ``pic_set_tiling`` (which never changes results: the current is
summed in integers), by coordinate descent from the default, and keeps the
fastest measured ms/step.  Timed windows span a multiple of every sort
interval so the sort cost is amortised fairly.  Results are cached in JSON
keyed by grid shape, particles per cell and solver; ``bench.py`` and
``workloads.build`` read the cache.

    python -m paper_1204_0838_amd.autotune --warmup 600 --steps 12
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")

DEFAULT = {"tile": (8, 8, 8), "guard": 1, "threads": 512, "interleave": 8, "sort_interval": 2}
SPACE = {
    "tile": [(8, 8, 8), (8, 8, 4), (8, 4, 4), (16, 8, 4), (16, 4, 4), (4, 4, 4), (16, 8, 8)],
    "guard": [0, 1, 2],
    "threads": [256, 512, 1024],
    "interleave": [1, 4, 8, 16],
    "sort_interval": [1, 2, 3, 4],
}


def key_of(cfg: dict) -> str:
    p = cfg["plasma"]["ppc"]
    return "{}x{}x{}|ppc{}|{}".format(*cfg["n"], p[0] * p[1] * p[2], cfg["solver"])


def lds_bytes(c: dict) -> int:
    T, g = c["tile"], c["guard"]
    fr = 1
    jr = 1
    for t in T:
        fr *= t + 2 * (g + 2)
        jr *= t + 2 * g + 5
    return 24 * jr + 24 * fr


def feasible(c: dict) -> bool:
    return lds_bytes(c) <= 160 * 1024


def time_candidate(sim, c: dict, steps: int) -> float:
    import torch

    sim.set_tiling(**c)
    sim.step(1)            # re-sort under the new tiling
    sim.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    sim.sync()
    return e0.elapsed_time(e1) / steps


def tune(sim, steps: int = 12, rounds: int = 2, log=sys.stderr):
    """Coordinate descent over SPACE; returns (best, table of (candidate, ms/step))."""
    best = dict(DEFAULT)
    seen = {}

    def measure(c):
        k = json.dumps(c, sort_keys=True)
        if k not in seen:
            seen[k] = time_candidate(sim, c, steps)
            if log:
                print(f"# tune {c} -> {seen[k]:.3f} ms/step", file=log, flush=True)
        return seen[k]

    best_ms = measure(best)
    for _ in range(rounds):
        improved = False
        for knob, values in SPACE.items():
            for v in values:
                c = dict(best)
                c[knob] = v
                if not feasible(c):
                    continue
                ms = measure(c)
                if ms < best_ms:
                    best, best_ms, improved = c, ms, True
        if not improved:
            break
    sim.set_tiling(**best)
    table = [(json.loads(k), ms) for k, ms in sorted(seen.items(), key=lambda kv: kv[1])]
    return best, best_ms, table


def load(cfg: dict, path: str = CACHE):
    """Cached best tiling for this workload shape, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    rec = cache.get(key_of(cfg))
    if not rec:
        return None
    best = dict(rec["best"])
    best["tile"] = tuple(best["tile"])
    return best


def save(cfg: dict, best: dict, best_ms: float, table, note: str, path: str = CACHE):
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[key_of(cfg)] = {"best": best, "ms_per_step": best_ms, "note": note,
                          "measured": [{"tiling": c, "ms_per_step": ms} for c, ms in table[:12]]}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=str, default="")
    ap.add_argument("--warmup", type=int, default=600)
    ap.add_argument("--steps", type=int, default=12)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1204_0838_amd import workloads

    cfg = workloads.C1
    if args.grid:
        cfg = workloads.scaled(cfg, [int(v) for v in args.grid.split(",")])
    sim = workloads.build(cfg, tuned=False)
    t0 = time.perf_counter()
    done = 0
    while done < args.warmup:
        k = min(100, args.warmup - done)
        sim.step(k)
        done += k
        print(f"# warm-up {done}/{args.warmup}", file=sys.stderr, flush=True)
    sim.sync()
    best, best_ms, table = tune(sim, args.steps)
    save(cfg, best, best_ms, table,
         f"coordinate descent at step {args.warmup} of the {cfg['name']} run, {args.steps} timed steps per candidate, "
         f"{time.perf_counter() - t0:.0f} s")
    print(json.dumps({"key": key_of(cfg), "best": best, "ms_per_step": best_ms}))


if __name__ == "__main__":
    main()
