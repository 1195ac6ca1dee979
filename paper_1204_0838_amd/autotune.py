"""Autotuner of the fused step's tiling: tile shape, drift guard, threads per
workgroup, in-tile interleave depth and sort interval.

It times ``pic_step`` on a live simulation for each candidate, switching the
tiling with ``pic_set_tiling`` (which never changes results: the current is
summed in integers).  The default search (tune_phases) times every one-knob
change of the default at several points of one run, since the cost of a
step changes over the run, combines the knobs that help and checks the
combination over a whole fresh run; ``--instant`` runs a coordinate descent
at one instant instead.  Timed windows span a multiple of every sort
interval so the sort cost is amortised fairly.  Results are cached in JSON
keyed by grid shape, particles per cell and solver; ``bench.py`` and
``workloads.build`` read the cache.

    python -m paper_1204_0838_amd.autotune --phases 150,450,750 --steps 12
    python -m paper_1204_0838_amd.autotune --instant --warmup 600 --steps 12
    python -m paper_1204_0838_amd.autotune --batch --warmup 60 --steps 6

The batched form tunes the members of a parameter scan per instance-size
class on the live batch (one tiling per class; threads per tile batch-wide).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")

DEFAULT = {"tile": (8, 8, 8), "guard": 1, "threads": 512, "interleave": 0, "sort_interval": 2}
SPACE = {
    "tile": [(8, 8, 8), (8, 8, 4), (8, 4, 4), (16, 8, 4), (16, 4, 4), (4, 4, 4), (16, 8, 8)],
    "guard": [0, 1, 2],
    "threads": [256, 512, 1024],
    "interleave": [0, 1, 8, 16],   # 0: level order, else the transpose depth
    "sort_interval": [1, 2, 3, 4],
}


def key_of(cfg: dict) -> str:
    p = cfg["plasma"]["ppc"]
    return "{}x{}x{}|ppc{}|{}".format(*cfg["n"], p[0] * p[1] * p[2], cfg["solver"])


def _pad_plane(p: int, m: int) -> int:
    # the tile kernel pads each LDS z-plane to 8 (mod m) words
    return p + ((8 - p % m) + m) % m


def lds_bytes(c: dict) -> int:
    T, g = c["tile"], c["guard"]
    f = [t + 2 * (g + 2) for t in T]
    j = [t + 2 * g + 5 for t in T]
    fr = _pad_plane(f[0] * f[1], 32) * f[2]
    jr = _pad_plane(j[0] * j[1], 16) * j[2]
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
    """Coordinate descent over SPACE; returns (best, ms/step, table of (candidate, ms/step)).

    The run evolves while it is tuned (the window moves, the wake grows), so
    each candidate is timed right after the current best, and it replaces the
    best only if it beats that fresh measurement by more than 1 %."""
    best = dict(DEFAULT)
    table = []
    best_ms = time_candidate(sim, best, steps)
    for _ in range(rounds):
        improved = False
        for knob, values in SPACE.items():
            for v in values:
                c = dict(best)
                c[knob] = v
                if c == best or not feasible(c):
                    continue
                ref = time_candidate(sim, best, steps)
                ms = time_candidate(sim, c, steps)
                table.append((c, ms, ref))
                if log:
                    print(f"# tune {c} -> {ms:.3f} ms/step (best now {ref:.3f})", file=log, flush=True)
                if ms < 0.99 * ref:
                    best, best_ms, improved = c, ms, True
                else:
                    best_ms = ref
        if not improved:
            break
    sim.set_tiling(**best)
    table.sort(key=lambda r: r[1] / r[2])
    return best, best_ms, [(c, ms) for c, ms, _ in table]


def knob_variants(base: dict) -> list:
    """Every one-knob change of `base` to another value of SPACE that fits LDS."""
    out = []
    for knob, values in SPACE.items():
        for v in values:
            c = dict(base)
            c[knob] = v
            if c != base and feasible(c):
                out.append(c)
    return out


def run_ms(cfg: dict, tiling: dict, steps: int, chunk: int = 20, jpost: str = "none") -> float:
    """Mean ms per step of a fresh run of `steps` steps from t = 0 with `tiling`."""
    import torch

    from . import workloads

    sim = workloads.build(cfg, tuned=False, jpost=jpost, **tiling)
    sim.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    total = 0.0
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        e0.record(sim.stream)
        sim.step(k)
        e1.record(sim.stream)
        sim.sync()
        total += e0.elapsed_time(e1)
        done += k
    sim.close()
    return total / steps


def tune_phases(cfg: dict, phases=(150, 450, 750), steps: int = 12, base_every: int = 3, log=sys.stderr,
                jpost: str = "none"):
    """Search over the whole run instead of one instant (the cost of a step
    changes as the wake forms and particles move).

    One run from t = 0 times, at each phase, every one-knob change of the
    default (knob_variants) for `steps` steps, each against a fresh timing of
    the default taken at most `base_every` candidates before it, as a ratio.
    Each knob keeps its value of least mean ratio over the phases if that is
    below 0.99; the knobs so chosen are combined, and the combination is kept
    only if a full fresh run with it is faster than one with the default.
    Returns (best, ms per step of best over the run, table of (candidate,
    mean ratio, per-phase ratios), note).  jpost: the current post-processing
    of the runs."""
    from . import workloads

    base = dict(DEFAULT)
    cands = knob_variants(base)
    ratios = {i: [] for i in range(len(cands))}
    sim = workloads.build(cfg, tuned=False, jpost=jpost, **base)
    done = 0
    for ph in phases:
        if ph < done:
            raise ValueError("phases overlap: the timings of one phase reach past the start of the next")
        while done < ph:
            k = min(100, ph - done)
            sim.step(k)
            done += k
        sim.sync()
        ref = None
        for i, c in enumerate(cands):
            if i % base_every == 0:
                ref = time_candidate(sim, base, steps)
                done += steps + 1
            ms = time_candidate(sim, c, steps)
            done += steps + 1
            ratios[i].append(ms / ref)
            if log:
                print(f"# phase {ph} (step {done}): {c} -> {ms:.3f} ms/step, default {ref:.3f}", file=log, flush=True)
    sim.close()
    table = []
    for i, c in enumerate(cands):
        r = ratios[i]
        table.append((c, sum(r) / len(r), r))
    best = dict(base)
    for knob in SPACE:
        rows = [(m, c) for c, m, _ in table if c[knob] != base[knob]]
        if rows:
            m, c = min(rows, key=lambda x: x[0])
            if m < 0.99:
                best[knob] = c[knob]
    if not feasible(best):
        best = min(table, key=lambda x: x[1])[0] if min(r[1] for r in table) < 0.99 else dict(base)
    total = int(cfg.get("steps", 1000))
    ms_base = run_ms(cfg, base, total, jpost=jpost)
    note = f"one-knob changes of the default timed at steps {list(phases)} of one run ({steps} steps each)"
    if best != base:
        ms_best = run_ms(cfg, best, total, jpost=jpost)
        if log:
            print(f"# whole run: default {ms_base:.3f}, combined {best} {ms_best:.3f} ms/step", file=log, flush=True)
        note += f"; whole {total}-step runs: combined {ms_best:.2f}, default {ms_base:.2f} ms per step"
        if ms_best >= ms_base:
            best, ms_best = dict(base), ms_base
            note += " (default kept)"
    else:
        ms_best = ms_base
        note += f"; no knob improved; whole run {ms_base:.2f} ms per step"
    table.sort(key=lambda r: r[1])
    return best, ms_best, table, note


def class_key(cls: str, cfg: dict) -> str:
    p = cfg["plasma"]["ppc"]
    return "batch|{}|ppc{}|{}".format(cls, p[0] * p[1] * p[2], cfg["solver"])


def time_batch(batch, steps: int) -> float:
    import torch

    batch.step(1)          # members re-sort under new tilings
    batch.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.step(steps)
    e1.record(batch.stream)
    batch.sync()
    return e0.elapsed_time(e1) / steps


def tune_batch(batch, sims, cfgs, steps: int = 6, rounds: int = 2, log=sys.stderr):
    """Per size-class coordinate descent on a live batch.

    Members of one class (workloads.size_class) share a tiling; threads per
    tile is one batch-wide knob (the batched tile launch uses one workgroup
    size).  As in tune(), each candidate is timed right after the current
    best.  Returns ({class: best tiling}, batch ms/step)."""
    from . import workloads

    classes = {}
    for i, c in enumerate(cfgs):
        classes.setdefault(workloads.size_class(c), []).append(i)
    best = {k: dict(DEFAULT) for k in classes}

    def measure(tilings):
        for k, idx in classes.items():
            for i in idx:
                sims[i].set_tiling(**tilings[k])
        return time_batch(batch, steps)

    best_ms = measure(best)
    if log:
        print(f"# batch tune start {best_ms:.3f} ms/step", file=log, flush=True)
    for _ in range(rounds):
        improved = False
        for knob, values in SPACE.items():
            for k in (classes if knob != "threads" else ["*"]):
                targets = list(classes) if k == "*" else [k]
                for v in values:
                    cand = {kk: dict(b) for kk, b in best.items()}
                    for t in targets:
                        cand[t][knob] = v
                    if cand == best or not all(feasible(cand[t]) for t in targets):
                        continue
                    ref = measure(best)
                    ms = measure(cand)
                    if log:
                        print(f"# batch tune {k} {knob}={v} -> {ms:.3f} ms/step (best now {ref:.3f})", file=log,
                              flush=True)
                    if ms < 0.99 * ref:
                        best, best_ms, improved = cand, ms, True
                    else:
                        best_ms = ref
        if not improved:
            break
    measure(best)
    return best, best_ms


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


def load_class(cls: str, cfg: dict, path: str = CACHE):
    """Cached tiling of a batch size class, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(class_key(cls, cfg))
    if not rec:
        return None
    best = dict(rec["best"])
    best["tile"] = tuple(best["tile"])
    return best


def save_classes(cfg: dict, best: dict, best_ms: float, note: str, path: str = CACHE):
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    for cls, b in best.items():
        cache[class_key(cls, cfg)] = {"best": b, "batch_ms_per_step": best_ms, "note": note}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)


def save(cfg: dict, best: dict, best_ms: float, table, note: str, path: str = CACHE):
    """table: (candidate, ms per step) or (candidate, mean ratio to the default, per-phase ratios)."""
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    rows = []
    for r in table[:16]:
        if len(r) == 2:
            rows.append({"tiling": r[0], "ms_per_step": r[1]})
        else:
            rows.append({"tiling": r[0], "ratio_to_default": round(r[1], 4),
                         "phase_ratios": [round(v, 4) for v in r[2]]})
    cache[key_of(cfg)] = {"best": best, "ms_per_step": best_ms, "note": note, "measured": rows}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=str, default="")
    ap.add_argument("--warmup", type=int, default=600)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--batch", action="store_true", help="tune the C3 parameter scan per size class")
    ap.add_argument("--instant", action="store_true",
                    help="coordinate descent at one instant (--warmup) instead of the whole-run search")
    ap.add_argument("--phases", type=str, default="150,450,750", help="steps of the run at which candidates are timed")
    ap.add_argument("--workload", choices=("c1", "c1p", "c4"), default="c1",
                    help="c4: the 2-ppc C1 geometry, tuned with the binomial filter standing in for the "
                         "denoiser (the tiling changes the particle phases only)")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1204_0838_amd import workloads

    if args.batch:
        cfgs = workloads.c3_members()
        sims, batch = workloads.build_batch(cfgs)
        t0 = time.perf_counter()
        batch.step(args.warmup)
        batch.sync()
        best, best_ms = tune_batch(batch, sims, cfgs, args.steps)
        save_classes(cfgs[0], best, best_ms, f"per-class coordinate descent on the live C3 batch at step "
                     f"{args.warmup}, {args.steps} timed batch steps per candidate, "
                     f"{time.perf_counter() - t0:.0f} s")
        print(json.dumps({"best": best, "batch_ms_per_step": best_ms}))
        return

    cfg = workloads.C1P if args.workload == "c1p" else workloads.C1
    jpost = "none"
    if args.workload == "c4":
        from paper_1204_0838_amd import c4

        cfg = c4.c4_config()
        jpost = "binomial"
    if args.grid:
        cfg = workloads.scaled(cfg, [int(v) for v in args.grid.split(",")])
    if not args.instant:
        t0 = time.perf_counter()
        best, best_ms, table, note = tune_phases(cfg, tuple(int(v) for v in args.phases.split(",")), args.steps,
                                                 jpost=jpost)
        if jpost != "none":
            note += f" (current post-processing: {jpost})"
        best["tile"] = list(best["tile"])
        save(cfg, best, best_ms, table, note + f", {time.perf_counter() - t0:.0f} s")
        print(json.dumps({"key": key_of(cfg), "best": best, "ms_per_step": best_ms}))
        return
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
