"""Named synthetic workloads shaped like the paper's laser-wakefield runs.

Configuration only (sizes, profiles, laser parameters); every step of the
simulation runs in the HIP library through ``paper_1204_0838_amd.pic``.

C1 is the 3D moving-window LWFA slab (C1P: the same inside a 16-cell
transverse perfectly matched layer): 512 x 256 x 256 cells, dx = 0.25 c/w_p
along the propagation axis with the perfect-dispersion solver at c dt = dx,
dy = dz = 0.5 c/w_p, 8 electrons per cell on a 2x2x2 lattice behind a
50-cell linear density ramp, and a y-polarised Gaussian laser (a0 = 4,
waist 5 c/w_p, intensity FWHM 2.5 / w_p) launched through the x boundary.
The paper resolves lambda0 with dx = 0.06 lambda0 (Section 3.1); keeping that
resolution gives lambda0 = 4.17 c/w_p, i.e. omega0 = 1.508 w_p.  The window
starts to move at c when the pulse peak reaches 64 cells from the front.

C2 is the quasi-cylindrical counterpart (two azimuthal modes): Nz = 4096,
Nr = 256, dz = 0.05, dr = 0.2 c/w_p, 32 particles per (z, r) cell at
uniform random azimuth over the radial cells below 252, the C1 laser on
mode 1 and the C1 density profile, c dt = dz / 2 (the window moves one cell
every second step once the pulse has entered), 2000 steps.

C3 is a parameter scan of 64 such setups of uneven size, advanced together
by the batched launcher: instance i draws from seeded stream 3 + i its grid
(nx uniform in 64..256, ny and nz in 32..64, each rounded to a multiple of
8 cells), its laser strength a0 in [2, 5] and its plateau density in
[0.5, 2] n0; spacings, solver, laser shape and ramp are C1's, the window
starts when the pulse peak is a quarter of the box from the front, 200 steps.
"""
from __future__ import annotations

import math

import numpy as np

C1 = {
    "name": "C1",
    "n": (512, 256, 256),
    "d": (0.25, 0.5, 0.5),
    "dt": 0.25,
    "solver": "pd",
    "steps": 1000,
    "plasma": {"x_start": 8.0, "ramp": 50.0, "n_plateau": 1.0, "ppc": (2, 2, 2)},
    "laser": {"a0": 4.0, "omega0": 2 * math.pi / (0.25 / 0.06), "waist": 5.0, "fwhm": 2.5, "t_peak": 10.0,
              "t_end": 20.0, "src_x": 2},
    "front_margin": 64,
}


# C1 inside the paper's transverse boundary: its 256 x 256-cell cross-section
# surrounded by a 16-cell perfectly matched layer on each side (Section 3.1),
# 512 x 288 x 288 cells; particles are loaded over the whole cross-section and
# those in the layer removed before their first push.
C1P = dict(C1, name="C1P", n=(512, 288, 288), pml=16)


C2 = {
    "name": "C2",
    "nz": 4096,
    "nr": 256,
    "dz": 0.05,
    "dr": 0.2,
    "dt": 0.025,
    "window_period": 2,
    "steps": 2000,
    "sort_interval": 16,
    "plasma": {"z_start": 2.0, "ramp": 12.5, "n_plateau": 1.0, "ppc": 32, "r_cells": 252, "seed": 5},
    "laser": {"a0": 4.0, "omega0": 2 * math.pi / (0.25 / 0.06), "waist": 5.0, "fwhm": 2.5, "t_peak": 10.0,
              "t_end": 20.0, "src_z": 2},
}


def c2_window_start(cfg: dict) -> int:
    """First step after which the C2 window moves: once the source is off."""
    return int(math.ceil(cfg["laser"]["t_end"] / cfg["dt"] - 1e-9))


def build_c2(cfg: dict = C2, capacity_factor: float = 1.05, device="cuda:0", sort_interval: int = 0,
             interleave: int = 0, threads: int = 0):
    """A CircSimulation holding the C2 workload at t = 0 (plasma loaded, laser and window set);
    sort_interval 0 takes the workload's (16: measured over the whole run against 2-32; most of the
    window is plasma at rest ahead of the pulse, which never leaves its tile)."""
    from .circ import CircSimulation

    p = cfg["plasma"]
    nz, nr = cfg["nz"], cfg["nr"]
    shifts = (cfg["steps"] - c2_window_start(cfg)) // cfg["window_period"] + 1
    cap = int(((nz - 2) * p["r_cells"] * p["ppc"]) * capacity_factor) + shifts * p["r_cells"] * p["ppc"]
    sim = CircSimulation(nz, nr, cfg["dz"], cfg["dr"], cfg["dt"], window_period=cfg["window_period"],
                         sort_interval=sort_interval or cfg.get("sort_interval", 0), max_particles=cap,
                         device=device, interleave=interleave, threads=threads)
    sim.add_empty_species(cap)
    sim.set_plasma(0, p["z_start"], p["ramp"], p["n_plateau"], p["ppc"], p["r_cells"], p["seed"])
    sim.inject_plasma(0, 0, nz - 2)
    L = cfg["laser"]
    sim.set_laser(L["a0"], L["omega0"], L["waist"], L["fwhm"], L["t_peak"], L["t_end"], L["src_z"])
    sim.set_window(c2_window_start(cfg))
    return sim


def scaled(cfg: dict, n) -> dict:
    """The same workload on a different grid (same spacings, profile and laser)."""
    out = dict(cfg)
    out["n"] = tuple(int(v) for v in n)
    return out


def window_start_step(cfg: dict) -> int:
    """Step at which the laser peak reaches `front_margin` cells from the front."""
    L = cfg["laser"]
    x_peak_cells = cfg["n"][0] - cfg["front_margin"] - L["src_x"]
    t = L["t_peak"] + x_peak_cells * cfg["d"][0]
    return max(int(math.ceil(L["t_end"] / cfg["dt"])), int(math.ceil(t / cfg["dt"])))


def initial_particles(cfg: dict) -> int:
    """Particles of the initial load (cells with n > 0 behind the injection margin)."""
    nx, ny, nz = cfg["n"]
    p = cfg["plasma"]
    ppc = p["ppc"][0] * p["ppc"][1] * p["ppc"][2]
    cells_x = max(0, (nx - 3) - int(math.ceil(p["x_start"])))
    return cells_x * ny * nz * ppc


def build(cfg: dict, capacity_factor: float = 1.05, device="cuda:0", tuned: bool = True, jpost: str = "none",
          species=None, **tiling):
    """A Simulation holding the workload at t = 0 (plasma loaded, laser and window set).

    species: optional list of (ppc lattice, density fraction), one electron
    species each on the same density profile (default: the configuration's
    lattice at the full density).  Tiling: explicit keyword arguments, else
    the autotuner's cached choice for this shape (when `tuned`), else the
    library defaults."""
    from . import autotune, pic

    if not tiling and tuned:
        tiling = autotune.load(cfg) or {}
    nx, ny, nz = cfg["n"]
    p = cfg["plasma"]
    if species is None:
        species = [(tuple(p["ppc"]), 1.0)]
    # every lattice slot of the window (the host-side bound of the initial load
    # counts them all) with headroom for electrons swept along with the window
    caps = []
    for lat, _ in species:
        ppc = lat[0] * lat[1] * lat[2]
        caps.append(int((nx - 3) * ny * nz * ppc * capacity_factor) + 4 * ny * nz * ppc)
    sim = pic.Simulation(cfg["n"], cfg["d"], cfg["dt"], solver=cfg["solver"], bc_x=1, max_particles=sum(caps),
                         device=device, jpost=jpost, **tiling)
    for s, ((lat, frac), cap) in enumerate(zip(species, caps)):
        sim.add_empty_species(cap)
        sim.set_plasma(s, p["x_start"], p["ramp"], p["n_plateau"] * frac, lat)
        sim.inject_plasma(s, 0, nx - 3)
    L = cfg["laser"]
    sim.set_laser(L["a0"], L["omega0"], L["waist"], L["fwhm"], L["t_peak"], L["t_end"], ny * cfg["d"][1] / 2,
                  nz * cfg["d"][2] / 2, L["src_x"])
    sim.set_window(window_start_step(cfg))
    if cfg.get("pml"):
        sim.set_pml(cfg["pml"])
    return sim


def c3_members(count: int = 64, seed0: int = 3, base: dict = C1) -> list:
    """Configurations of the C3 parameter-scan instances (see the module doc)."""
    from .inputs import uniform53

    out = []
    for i in range(count):
        u = uniform53(seed0 + i, np.arange(5, dtype=np.uint64))
        nx = 64 + int(u[0] * 193)
        ny = 32 + int(u[1] * 33)
        nz = 32 + int(u[2] * 33)
        n = tuple(8 * int(round(v / 8.0)) for v in (nx, ny, nz))
        cfg = scaled(base, n)
        cfg["name"] = f"C3[{i}]"
        cfg["steps"] = 200
        cfg["laser"] = dict(base["laser"], a0=2.0 + 3.0 * float(u[3]))
        cfg["plasma"] = dict(base["plasma"], n_plateau=0.5 + 1.5 * float(u[4]))
        cfg["front_margin"] = n[0] // 4
        out.append(cfg)
    return out


def size_class(cfg: dict) -> str:
    """Instance-size class used to share autotuned tilings across a scan."""
    nx, ny, nz = cfg["n"]
    cells = nx * ny * nz
    return "S" if cells < (1 << 18) else ("M" if cells < (1 << 19) else "L")


def build_batch(cfgs: list, capacity_factor: float = 1.3, device="cuda:0", tilings=None):
    """Simulations for every configuration plus the Batch that drives them.

    tilings: optional list (one dict per member) of tiling keywords."""
    from . import pic

    sims = []
    for i, cfg in enumerate(cfgs):
        t = dict(tilings[i]) if tilings else {}
        sims.append(build(cfg, capacity_factor, device, tuned=False, **t))
    return sims, pic.Batch(sims)
