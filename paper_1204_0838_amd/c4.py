"""Learned current denoiser at few particles per cell against the plain
binomial-filtered run at many, on the C1 laser-wakefield geometry.

Steps (every one runs through the HIP library; torch only moves crops):

The denoiser's output is J' = B(J + sigma curl(y)): the binomial filter of
the current plus a divergence-free learned correction, so the denoised
current keeps the filtered current's charge balance and, like it, carries
no grid-scale (Nyquist) modes.

1. Training pairs, exactly aligned: one high-ppc run whose plasma is two
   electron species on the same fields, the 32-ppc lattice (4x4x2) at 15/16
   of the density and the 2-ppc lattice (1x1x2) at 1/16.  At a sampled step
   the split path pushes both species and deposits the 2-ppc one first: 16 x
   its current is exactly what a 2-ppc run deposits from this state (the
   input); after the other species and the field step, J holds the filtered
   total current of the same step (the target).  Seeded crops of the window
   give the pairs; every other step is the fused production step.  (A 2-ppc
   run advanced beside a 32-ppc run instead drifts to another state, and its
   current then differs from the target by more than sampling noise.)
2. Training: Adam on the matrix cores (pic_dn_trainer), per-component scale
   = RMS of the targets.
2b. Optional rollout pairs (--rollout-steps N): pairs from the states the
   denoised run itself visits, then further training from the trained
   parameters.  One run carries the 2-ppc lattice at full density, whose
   current, denoised, drives the fields (the denoised 2-ppc run), and the
   32-ppc lattice at full density as passive particles pushed by the same
   fields: at every step the split path pushes both species and deposits
   the 2-ppc one (J_A, the input), and the field step runs on J_A alone; at
   sampled steps the passive species is deposited too (J_A + J_B) and the
   binomial filter of J_B, computed by the library on a particle-free grid
   of the same shape, is the target.
3. Evaluation: a 2-ppc run with the trained denoiser (fused step) and a
   2-ppc run with the binomial filter, both compared with the 32-ppc run on
   the wake field E_x over the whole window at fixed checkpoints; a second
   32-ppc run on another sub-cell lattice (2x4x4) gives the noise floor of
   that comparison.  Throughput: wall-clock steps per second on the same
   grid (the runs carry 16x different particle counts).

    python -m paper_1204_0838_amd.c4 --out c4_out                 # full C1 grid, 1000 steps
    python -m paper_1204_0838_amd.c4 --grid 128,64,64 --steps 200  # small rehearsal
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

PPC32 = (4, 4, 2)
PPC32_ALT = (2, 4, 4)
PPC2 = (1, 1, 2)


def _log(msg):
    print(f"# [{time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _cfg(base, ppc):
    cfg = dict(base)
    cfg["plasma"] = dict(base["plasma"], ppc=tuple(ppc))
    return cfg


def c4_config():
    """The C4 workload: the C1 geometry at 2 particles per cell."""
    from . import workloads

    return _cfg(workloads.C1, PPC2)


def _ex_window(sim):
    """E_x in window order (x index 0 = the window's trailing cell), host float32."""
    import torch

    _, org = sim.window_state()
    return torch.roll(sim.E[0], shifts=-org, dims=2).cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-30))


def collect_pairs(base, steps, sample_steps, crop, ncrops, seed, axis_share=0.75):
    """Aligned pairs from the two-species high-ppc run (see the module doc)
    and the plain 32-ppc run's E_x checkpoints, ms per step and particles.
    A share `axis_share` of the crops contains the laser axis, where the
    wake and the strongest currents are (a uniform draw would put it in a
    few percent of them); the rest are uniform over the window."""
    import torch

    from . import workloads

    mixed = workloads.build(_cfg(base, PPC32), jpost="binomial", species=[(PPC32, 15.0 / 16.0), (PPC2, 1.0 / 16.0)])
    nx, ny, nz = base["n"]
    cx, cy, cz = crop
    rng = np.random.default_rng(seed)
    per = int(math.ceil(ncrops / max(1, len(sample_steps))))
    pairs = []
    t0 = time.perf_counter()
    for st in range(1, steps + 1):
        if st in sample_steps and len(pairs) < ncrops:
            _, org = mixed.window_state()   # the step's current is deposited in the frame before its window shift
            mixed.gather_push(0)
            mixed.gather_push(1)
            mixed.deposit(1)
            js = 16.0 * torch.roll(mixed.J, shifts=-org, dims=3)
            mixed.deposit(0)
            mixed.field_step()
            jb = torch.roll(mixed.J, shifts=-org, dims=3)
            for _ in range(per):
                if len(pairs) >= ncrops:
                    break
                x0 = int(rng.integers(0, nx - cx + 1))
                if rng.random() < axis_share:   # a crop that contains the laser axis (the wake)
                    y0 = min(max(ny // 2 - cy // 2 + int(rng.integers(-(cy // 4), cy // 4 + 1)), 0), ny - cy)
                    z0 = min(max(nz // 2 - cz // 2 + int(rng.integers(-(cz // 4), cz // 4 + 1)), 0), nz - cz)
                else:
                    y0 = int(rng.integers(0, ny - cy + 1))
                    z0 = int(rng.integers(0, nz - cz + 1))
                sl = (slice(None), slice(z0, z0 + cz), slice(y0, y0 + cy), slice(x0, x0 + cx))
                pairs.append((js[sl].contiguous(), jb[sl].contiguous()))
        else:
            mixed.step(1)
        if st % 50 == 0:
            _log(f"pairs run step {st}/{steps}, {len(pairs)} crops, {time.perf_counter() - t0:.0f} s")
    mixed.close()
    ex32, ms32, n32, _ = run_eval(base, PPC32, "binomial", steps)
    return pairs, ex32, ms32, n32


def collect_rollout_pairs(base, steps, sample_steps, crop, ncrops, seed, params, scale, axis_share=0.75):
    """Aligned pairs from the denoised 2-ppc run's own states (see the module doc, 2b)."""
    import torch

    from . import pic, workloads

    sim = workloads.build(_cfg(base, PPC32), jpost="denoiser", species=[(PPC2, 1.0), (PPC32, 1.0)])
    sim.set_denoiser(params, scale)
    filt = pic.Simulation(base["n"], base["d"], base["dt"], solver=base["solver"], bc_x=1, jpost="binomial",
                          max_particles=1)
    nx, ny, nz = base["n"]
    cx, cy, cz = crop
    rng = np.random.default_rng(seed)
    per = int(math.ceil(ncrops / max(1, len(sample_steps))))
    pairs = []
    t0 = time.perf_counter()
    for st in range(1, steps + 1):
        _, org = sim.window_state()
        sim.gather_push(0)
        sim.gather_push(1)
        sim.deposit(0)
        ja = sim.J.clone()                     # the 2-ppc run's own current
        if st in sample_steps and len(pairs) < ncrops:
            sim.deposit(1)                     # + the passive 32-ppc particles
            with torch.no_grad():              # J_B in window order: the filter grid's window has origin 0
                filt.J.copy_(torch.roll(sim.J - ja, shifts=-org, dims=3))
            filt.current_filter()              # the library's binomial filter of J_B
            js = torch.roll(ja, shifts=-org, dims=3)
            jb = filt.J
            for _ in range(per):
                if len(pairs) >= ncrops:
                    break
                x0 = int(rng.integers(0, nx - cx + 1))
                if rng.random() < axis_share:
                    y0 = min(max(ny // 2 - cy // 2 + int(rng.integers(-(cy // 4), cy // 4 + 1)), 0), ny - cy)
                    z0 = min(max(nz // 2 - cz // 2 + int(rng.integers(-(cz // 4), cz // 4 + 1)), 0), nz - cz)
                else:
                    y0 = int(rng.integers(0, ny - cy + 1))
                    z0 = int(rng.integers(0, nz - cz + 1))
                sl = (slice(None), slice(z0, z0 + cz), slice(y0, y0 + cy), slice(x0, x0 + cx))
                pairs.append((js[sl].contiguous(), jb[sl].contiguous()))
        with torch.no_grad():
            sim.J.copy_(ja)                    # the fields see the denoised 2-ppc current only
        sim.field_step()
        if st % 50 == 0:
            _log(f"rollout run step {st}/{steps}, {len(pairs)} crops, {time.perf_counter() - t0:.0f} s")
    sim.close()
    filt.close()
    return pairs


def binomial_init(rng, noise=0.3):
    """Parameters whose network output is the binomial filter: J' = B(J).

    The last layer starts at zero (y = 0, so J' = B(J) exactly); the first
    two layers start random, giving training features to build on."""
    W1 = noise * rng.standard_normal((32, 3, 3, 3, 3)) / np.sqrt(81.0)
    W2 = noise * rng.standard_normal((32, 32, 3, 3, 3)) / np.sqrt(864.0)
    W3 = np.zeros((3, 32, 3, 3, 3))
    return [W1, np.zeros(32), W2, np.zeros(32), W3, np.zeros(3)]


def train(pairs, crop, cell, epochs, lr, seed, batch=8, start=None, start_scale=None):
    """Adam on mini-batches of crops, starting from the binomial filter,
    with the biases held at zero.

    A seeded tenth of the crops is held out; the parameters with the lowest
    held-out loss are kept, and the binomial start itself if training never
    beats it.  Returns (params, scale, history)."""
    from . import pic

    tgt_rms = np.sqrt(np.mean([[float((t[d] ** 2).mean()) for d in range(3)] for _, t in pairs], axis=0))
    scale = np.maximum(tgt_rms, 1e-12).astype(np.float32) if start_scale is None else start_scale
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(pairs))
    nval = max(1, len(pairs) // 10)
    val = [pairs[i] for i in order[:nval]]
    trn = [pairs[i] for i in order[nval:]]
    P = binomial_init(rng) if start is None else [np.asarray(a) for a in start]
    tr = pic.DenoiserTrainer(crop, cell=cell)
    tr.set_params(P, scale)
    tr.freeze_biases(True)     # zero biases: no correction where J = 0, and net(a J) = a net(J)

    def val_loss():
        return tr.eval([p[0] for p in val], [p[1] for p in val])

    init = val_loss()
    best, best_params = init, tr.get_params()
    hist = {"val_loss_binomial_start" if start is None else "val_loss_start": init, "val_loss": [], "train_loss": []}
    nstep = epochs * ((len(trn) + batch - 1) // batch)
    k = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(len(trn))
        tl = []
        for b0 in range(0, len(trn), batch):
            idx = perm[b0:b0 + batch]
            frac = k / max(1, nstep)
            cur = lr if frac < 0.6 else (lr * 0.3 if frac < 0.85 else lr * 0.1)
            tl.append(tr.step_batch([trn[i][0] for i in idx], [trn[i][1] for i in idx], cur))
            k += 1
        v = val_loss()
        hist["train_loss"].append(float(np.mean(tl)))
        hist["val_loss"].append(v)
        if v < best:
            best, best_params = v, tr.get_params()
        _log(f"epoch {ep + 1}/{epochs}: train {hist['train_loss'][-1]:.5f}, held-out {v:.5f} "
             f"({'binomial start' if start is None else 'start'} {init:.5f}), {time.perf_counter() - t0:.0f} s")
    hist["kept"] = "trained" if best < init else ("binomial start" if start is None else "start")
    hist["val_loss_kept"] = best
    tr.close()
    return best_params, scale, hist


def run_eval(base, ppc, jpost, steps, params=None, scale=None, continuity=False):
    """One run; returns (E_x checkpoints, ms/step, particles, extra)."""
    import torch

    from . import workloads

    sim = workloads.build(_cfg(base, ppc), jpost=jpost, tuned=(ppc == PPC32))
    if params is not None:
        sim.set_denoiser(params, scale)
    checkpoints = sorted(set(range(100, steps + 1, 100)) | {steps})
    ex = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ms = 0.0
    done = 0
    t0 = time.perf_counter()
    for cp in checkpoints:
        k = cp - done
        if continuity and cp == checkpoints[-1]:
            k -= 1
        e0.record(sim.stream)
        sim.step(k)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        done += k
        if not (continuity and cp == checkpoints[-1]):
            ex[cp] = _ex_window(sim)
        _log(f"{jpost} ppc {ppc} step {done}/{steps}, {time.perf_counter() - t0:.0f} s")
    extra = {}
    if continuity:
        # last step by the split path, to measure the continuity residual of the post-processed current
        sim.gather_push(0)
        sim.deposit(0)
        raw = sim.J.clone()
        sim.current_filter()
        r, jm = sim.continuity(0)
        extra = {"continuity_residual": r, "max_abs_J": jm, "ratio": r / jm if jm > 0 else None}
        sim.J.copy_(raw)           # the field step applies the post-processing itself
        sim.field_step()
        done += 1
        ex[steps] = _ex_window(sim)
    n = sim.reduce()["n_particles"]
    sim.close()
    return ex, ms / (done - (1 if continuity else 0)), n, extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=str, default="")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--crops", type=int, default=256)
    ap.add_argument("--crop", type=str, default="128,64,64")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--out", type=str, default="c4_out")
    ap.add_argument("--no-floor", action="store_true", help="skip the second 32-ppc run (noise floor)")
    ap.add_argument("--axis-share", type=float, default=0.75, help="share of training crops containing the laser axis")
    ap.add_argument("--rollout-steps", type=int, default=0,
                    help="steps of the denoised run whose states give a second set of pairs (0: none)")
    ap.add_argument("--rollout-epochs", type=int, default=4)
    ap.add_argument("--alphas", type=str, default="",
                    help="also evaluate the learned correction scaled by each of these factors (comma list)")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1204_0838_amd import workloads

    base = workloads.C1
    if args.grid:
        base = workloads.scaled(base, [int(v) for v in args.grid.split(",")])
    crop = tuple(int(v) for v in args.crop.split(","))
    os.makedirs(args.out, exist_ok=True)
    steps = args.steps
    sample_steps = set(np.linspace(steps // 20, steps - 1, 24).astype(int).tolist())
    _log(f"grid {base['n']}, {steps} steps, pairs from steps {min(sample_steps)}..{max(sample_steps)}")
    pairs, ex32, ms32, n32 = collect_pairs(base, steps, sample_steps, crop, args.crops, seed=5,
                                           axis_share=args.axis_share)
    _log(f"{len(pairs)} training pairs; 32-ppc run {ms32:.1f} ms/step, {n32} particles")
    t_train = time.perf_counter()
    params, scale, hist = train(pairs, crop, base["d"], args.epochs, args.lr, seed=6, batch=args.batch)
    del pairs
    hist_rollout = None
    if args.rollout_steps > 0:
        rs = args.rollout_steps
        rsample = set(np.linspace(max(1, rs // 10), rs - 1, 16).astype(int).tolist())
        rpairs = collect_rollout_pairs(base, rs, rsample, crop, args.crops // 2, seed=7, params=params, scale=scale,
                                       axis_share=args.axis_share)
        _log(f"{len(rpairs)} rollout pairs from steps {min(rsample)}..{max(rsample)}")
        params, scale, hist_rollout = train(rpairs, crop, base["d"], args.rollout_epochs, args.lr * 0.3, seed=8,
                                            batch=args.batch, start=params, start_scale=scale)
        del rpairs
    t_train = time.perf_counter() - t_train
    np.savez(os.path.join(args.out, "denoiser_params.npz"), W1=params[0], b1=params[1], W2=params[2], b2=params[3],
             W3=params[4], b3=params[5], scale=scale)
    exd, msd, nd, cont = run_eval(base, PPC2, "denoiser", steps, params, scale, continuity=True)
    exb, msb, nb, _ = run_eval(base, PPC2, "binomial", steps)
    scaled = {}
    for a in [float(v) for v in args.alphas.split(",") if v.strip()]:
        pa = [params[0], params[1], params[2], params[3], a * np.asarray(params[4]), a * np.asarray(params[5])]
        exa, _, _, _ = run_eval(base, PPC2, "denoiser", steps, pa, scale)
        scaled[str(a)] = {str(k): _rel(exa[k], ex32[k]) for k in sorted(exa)}
    floor = None
    if not args.no_floor:
        exf, msf, nf, _ = run_eval(base, PPC32_ALT, "binomial", steps)
        floor = {str(k): _rel(exf[k], ex32[k]) for k in sorted(exf)}
    out = {
        "grid": list(base["n"]), "steps": steps, "crop": list(crop), "crops": args.crops,
        "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "axis_share": args.axis_share,
        "train_seconds": t_train, "training": hist, "rollout_training": hist_rollout,
        "rollout_steps": args.rollout_steps,
        "scale": scale.tolist(),
        "ms_per_step": {"ppc32_binomial": ms32, "ppc2_denoiser": msd, "ppc2_binomial": msb},
        "particles": {"ppc32": n32, "ppc2_denoiser": nd, "ppc2_binomial": nb},
        "speedup_steps_per_s_denoised_vs_ppc32": ms32 / msd,
        "wake_ex_rel_l2_vs_ppc32": {
            "ppc2_denoiser": {str(k): _rel(exd[k], ex32[k]) for k in sorted(exd)},
            "ppc2_binomial": {str(k): _rel(exb[k], ex32[k]) for k in sorted(exb)},
            "ppc32_other_lattice_noise_floor": floor,
            "ppc2_denoiser_correction_scaled": scaled,
        },
        "denoised_continuity": cont,
    }
    with open(os.path.join(args.out, "c4_summary.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
