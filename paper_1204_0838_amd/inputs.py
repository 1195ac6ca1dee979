"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws numbers and lays them out; it holds none of the
particle-in-cell arithmetic (no shapes, no push, no deposit, no field update).
Both sides of every parity check read the arrays it returns, so they start
from bit-identical states: positions are an int32 cell index plus an FP32
in-cell offset in [0, 1), momenta and weights are FP32.

Random draws use SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) in counter mode: draw ``k`` of
stream ``seed`` is ``mix64(seed * G + (k + 1) * G)`` with G the 64-bit golden
ratio increment; uniforms keep the top 53 bits.  Gaussians use Box-Muller.

Units are the plasma-normalised ones of the paper's runs: lengths in c/w_p,
times in 1/w_p, momenta u = p/(m_e c) (so c = 1), densities in n0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_G = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# electron rest energy in eV: converts a temperature in eV to a thermal spread of u
ME_C2_EV = 510998.95


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output for ``counters`` (uint64 array) of stream ``seed``."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) * _G + (counters.astype(np.uint64) + np.uint64(1)) * _G
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform53(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits."""
    return (splitmix64(seed, counters) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def offset_f32(u: np.ndarray) -> np.ndarray:
    """Round a uniform in [0,1) toward zero onto the 2^-24 lattice (exact in FP32, < 1)."""
    return (np.floor(u * 2.0 ** 24) * 2.0 ** -24).astype(np.float32)


@dataclass
class Grid:
    n: tuple            # cells (nx, ny, nz), x = propagation axis, x fastest in memory
    d: tuple            # cell sizes (c/w_p)
    dt: float           # time step (1/w_p)
    solver: str = "yee"  # "yee" or "pd"
    window: bool = False  # moving window along x (else periodic in x)

    @property
    def ncells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclass
class Particles:
    cell: np.ndarray     # int32 [np], linear cell index i + nx*(j + ny*k)
    off: np.ndarray      # float32 [3, np], in-cell offsets in [0, 1)
    u: np.ndarray        # float32 [3, np], u = gamma v / c
    w: np.ndarray        # float32 [np], density weight n/ppc
    id: np.ndarray       # int32 [np]
    q: float = -1.0
    m: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def count(self) -> int:
        return int(self.cell.shape[0])

    def positions(self, grid: Grid) -> np.ndarray:
        """Absolute positions (FP64, [3, np]) of the stored (cell, offset) pairs."""
        nx, ny, _ = grid.n
        c = self.cell.astype(np.int64)
        idx = (c % nx, (c // nx) % ny, c // (nx * ny))
        return np.stack([(idx[a] + self.off[a].astype(np.float64)) * grid.d[a] for a in range(3)])


def c0_grid() -> Grid:
    """64x32x32 periodic cells of 0.2 c/w_p; Courant number 0.5 of the 3D Yee limit."""
    d = 0.2
    return Grid(n=(64, 32, 32), d=(d, d, d), dt=0.5 * d / math.sqrt(3.0), solver="yee")


def uniform_random_plasma(grid: Grid, ppc: int, seed: int, temperature_ev: float = 10.0,
                          ux_amp: float = 0.01, density: float = 1.0) -> Particles:
    """Uniform plasma, ``ppc`` electrons per cell at seeded uniform offsets.

    Momenta: Gaussian of spread sqrt(T/(m c^2)) per component plus a
    sinusoidal x-perturbation ``ux_amp * sin(2 pi x / Lx)``.
    Draw counter of particle p, draw r is ``8 p + r`` (r = 0..5).
    """
    nx, ny, nz = grid.n
    ncell = grid.ncells
    npart = ncell * ppc
    p = np.arange(npart, dtype=np.uint64)
    cell = (np.arange(npart, dtype=np.int64) // ppc).astype(np.int32)
    off = np.stack([offset_f32(uniform53(seed, p * np.uint64(8) + np.uint64(r))) for r in range(3)])
    sigma = math.sqrt(temperature_ev / ME_C2_EV)
    g = []
    for r in (3, 4, 5):
        u1 = uniform53(seed, p * np.uint64(8) + np.uint64(r))
        u2 = uniform53(seed ^ 0x5DEECE66D, p * np.uint64(8) + np.uint64(r))
        g.append(np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2))
    ix = cell.astype(np.int64) % nx
    x = (ix + off[0].astype(np.float64)) * grid.d[0]
    lx = nx * grid.d[0]
    ux = sigma * g[0] + ux_amp * np.sin(2.0 * math.pi * x / lx)
    u = np.stack([ux, sigma * g[1], sigma * g[2]]).astype(np.float32)
    w = np.full(npart, density / ppc, dtype=np.float32)
    return Particles(cell=cell, off=off, u=u, w=w, id=np.arange(npart, dtype=np.int32),
                     meta={"seed": seed, "ppc": ppc, "sigma_u": sigma})


def lattice_plasma(grid: Grid, per_dim=(2, 2, 2), density: float = 1.0,
                   ux_amp: float = 0.0, mode: int = 1) -> Particles:
    """Quiet-start plasma: per_dim sub-cell lattice points per cell at offsets (k + 1/2)/n.

    Optional cold x-momentum mode ``ux_amp * sin(2 pi mode x / Lx)``.
    """
    nx, ny, nz = grid.n
    ppc = per_dim[0] * per_dim[1] * per_dim[2]
    sub = [(np.arange(n) + 0.5) / n for n in per_dim]
    sx, sy, sz = np.meshgrid(sub[0], sub[1], sub[2], indexing="ij")
    sub_off = np.stack([sx.ravel(), sy.ravel(), sz.ravel()])          # [3, ppc]
    npart = grid.ncells * ppc
    cell = (np.arange(npart, dtype=np.int64) // ppc).astype(np.int32)
    k = np.arange(npart) % ppc
    off = sub_off[:, k].astype(np.float32)
    ix = cell.astype(np.int64) % nx
    x = (ix + off[0].astype(np.float64)) * grid.d[0]
    lx = nx * grid.d[0]
    u = np.zeros((3, npart), dtype=np.float32)
    u[0] = (ux_amp * np.sin(2.0 * math.pi * mode * x / lx)).astype(np.float32)
    w = np.full(npart, density / ppc, dtype=np.float32)
    return Particles(cell=cell, off=off, u=u, w=w, id=np.arange(npart, dtype=np.int32),
                     meta={"ppc": ppc, "lattice": per_dim})


def c0_particles(seed: int = 1) -> Particles:
    """The uniform 8-ppc, 10 eV, 0.01c-perturbed electron plasma on the 64x32x32 grid."""
    return uniform_random_plasma(c0_grid(), ppc=8, seed=seed)


def random_fields(grid: Grid, seed: int, amp: float = 1.0) -> np.ndarray:
    """Seeded uniform(-amp, amp) FP32 values for E and B: array [6, nz, ny, nx]."""
    nx, ny, nz = grid.n
    k = np.arange(6 * grid.ncells, dtype=np.uint64)
    v = (2.0 * uniform53(seed, k) - 1.0) * amp
    return v.astype(np.float32).reshape(6, nz, ny, nx)
