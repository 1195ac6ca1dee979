"""Run diagnostics along the C1 laser-wakefield run, of the kind Section 3.2
reports for the paper's runs (Fig. 1: length of the accelerating phase on
axis, collection phase space; Table 1: charge, energy and normalised
emittance of the accelerated bunch; Figs. 3-4: spectra), on the synthetic
C1 workload.  Every quantity is computed on the device by the library's
diagnostic calls; this module only schedules them and prints the series.

    python -m paper_1204_0838_amd.lwfa_diag --steps 1000 --every 100

At each checkpoint: the laser centroid (window coordinates, from the
transverse field energy), the accelerating-phase length on axis behind it,
the beam of electrons with u_x > ux_min (count, charge, mean u_x,
emittances), the peak of the kinetic-energy spectrum of that beam, and the
time each call took (wall clock around the synchronising call) with the
bytes it streams.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import workloads


def _timed(fn, *a, **k):
    t0 = time.perf_counter()
    r = fn(*a, **k)
    return r, (time.perf_counter() - t0) * 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--ux-min", type=float, default=3.0, help="u_x threshold of the accelerated beam (m_e c)")
    ap.add_argument("--grid", type=str, default="")
    args = ap.parse_args()
    cfg = workloads.C1
    if args.grid:
        cfg = workloads.scaled(cfg, [int(v) for v in args.grid.split(",")])
    sim = workloads.build(cfg)
    d = cfg["d"]
    ncell = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    series = []
    done = 0
    while done < args.steps:
        k = min(args.every, args.steps - done)
        sim.step(k)
        done += k
        sim.sync()
        npart = sim.reduce()["n_particles"]
        fm, t_fm = _timed(sim.field_moments, True)
        x_laser = fm[1] / fm[0] if fm[0] > 0 else 0.0
        lacc, t_line = _timed(sim.accelerating_length, x_laser)
        beam, t_beam = _timed(sim.beam_moments, 0, args.ux_min)
        (charge, _), t_spec = _timed(sim.spectrum, 0, 0, 0.0, 100.0, 200)
        ids, x, ux, nsel, = sim.select_particles(0, args.ux_min, cap=1 << 16)
        shift, _ = sim.window_state()
        peak = float((np.argmax(charge) + 0.5) * 0.5) if charge.sum() > 0 else 0.0
        rec = {"step": done, "window_shift": shift, "laser_centroid": x_laser, "laser_energy": fm[0],
               "accelerating_length": lacc, "beam_count": beam["count"], "beam_charge": beam["charge"],
               "beam_mean_ux": beam["mean_ux"], "eps_ny": beam["eps_ny"], "eps_nz": beam["eps_nz"],
               "spectrum_peak_gamma_minus_1": peak, "selected": nsel,
               "ms": {"field_moments": t_fm, "axis_line+length": t_line, "beam_moments": t_beam,
                      "spectrum": t_spec},
               "particles": npart,
               # bytes streamed: E, B per cell; cell + u_x per particle and
               # off_y, off_z, u_y, u_z, w per selected one; cell, u, w per particle
               "GB_per_s": {"field_moments": 24.0 * ncell / (t_fm * 1e6),
                            "beam_moments": (8.0 * npart + 20.0 * beam["count"]) / (t_beam * 1e6),
                            "spectrum": 20.0 * npart / (t_spec * 1e6)}}
        series.append(rec)
        print(f"# step {done}: laser at {x_laser:.2f}, accelerating phase {lacc:.2f} c/wp, beam "
              f"{beam['count']} (u_x > {args.ux_min}), eps_y {beam['eps_ny']:.3f}, eps_z {beam['eps_nz']:.3f} c/wp",
              file=sys.stderr, flush=True)
    print(json.dumps({"workload": "C1", "ux_min": args.ux_min, "series": series}))


if __name__ == "__main__":
    main()
