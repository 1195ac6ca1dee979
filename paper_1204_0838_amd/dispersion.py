"""Laser group velocity under the Yee and the perfect-dispersion solvers.

Section 3.3 of the paper attributes the differences between its normal- and
perfect-dispersion runs to the numerical slowdown of the laser pulse in the
Yee scheme (Section 1: the FDTD scheme's axial dispersion error lowers the
pulse's group velocity), which the perfect-dispersion curl removes along
the propagation axis (Section 2).  This module measures it directly: the
C1 laser is launched through the x boundary of a grid with the C1 cell
sizes, and the centroid of its electromagnetic energy (pic_field_moments,
transverse components) is followed in time after the source has switched
off; a least-squares line through the centroids gives the pulse's group
velocity.  Both solvers run the same pulse: Yee at 0.98 of its 3D Courant
limit, perfect dispersion at c dt = dx.  (In the C1 plasma, which is
near-critical for the pulse, the field-energy centroid also carries the
wake's and the scattered light's fields and does not follow the pulse; the
measurement is made in vacuum.)

    python -m paper_1204_0838_amd.dispersion            # C1 grid, vacuum

Every step runs in the HIP library; this module only sets runs up and fits
the line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import pic, workloads


def yee_dt(d, courant=0.98):
    return courant / math.sqrt(sum(1.0 / (v * v) for v in d))


def measure(solver, n=None, d=None, waist=None, t_from=30.0, t_to=110.0, every=5, device="cuda:0"):
    """Centroid velocity of the C1 laser pulse in vacuum on a grid of n cells of d.

    Returns dict(v_g, residual, times, centroids, dt, steps, field_ms_per_step).
    The source plane is the C1 one; the transverse profile is C1's waist
    unless `waist` is given (1e12: a plane wave)."""
    cfg = workloads.C1
    n = tuple(n or cfg["n"])
    d = tuple(d or cfg["d"])
    dt = d[0] if solver == "pd" else yee_dt(d)
    L = dict(cfg["laser"])
    if waist is not None:
        L["waist"] = waist
    sim = pic.Simulation(n, d, dt, solver=solver, bc_x=1, max_particles=16, device=device)
    sim.add_empty_species(16)
    sim.set_laser(L["a0"], L["omega0"], L["waist"], L["fwhm"], L["t_peak"], L["t_end"], n[1] * d[1] / 2,
                  n[2] * d[2] / 2, L["src_x"])
    ts, xc = [], []
    step = 0
    total = int(round(t_to / dt))
    sim.profile_enable(True)
    while step < total:
        sim.step(1)
        step += 1
        t = step * dt
        if t >= t_from and step % every == 0:
            m = sim.field_moments(transverse_only=True)    # synchronises
            ts.append(t)
            xc.append(m[1] / m[0])
    prof = sim.profile_read()
    sim.close()
    ts, xc = np.array(ts), np.array(xc)
    coef = np.polyfit(ts, xc, 1)
    res = np.abs(xc - np.polyval(coef, ts)).max()
    return {"solver": solver, "v_g": float(coef[0]), "residual": float(res), "dt": dt, "steps": total,
            "times": ts.tolist(), "centroids": xc.tolist(), "field_ms_per_step": prof["field_ms"] / max(1, total),
            "ms_per_step": sum(prof[k] for k in ("sort_ms", "tile_ms", "loose_ms", "jpost_ms", "field_ms",
                                                 "window_ms")) / max(1, total)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=str, default="", help="nx,ny,nz (default: the C1 grid)")
    args = ap.parse_args()
    n = tuple(int(v) for v in args.grid.split(",")) if args.grid else None
    out = {}
    for solver in ("pd", "yee"):
        t0 = time.perf_counter()
        r = measure(solver, n=n)
        r.pop("times")
        r.pop("centroids")
        out[solver] = r
        print(f"# {solver}: v_g {r['v_g']:.6f} (fit residual {r['residual']:.2e} c/wp), field update "
              f"{r['field_ms_per_step']:.3f} ms/step, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    out["slowdown"] = out["pd"]["v_g"] - out["yee"]["v_g"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
