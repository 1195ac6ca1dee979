"""Python access to the FP64 quasi-cylindrical (m = 0, 1) reference in circ.c.

TEST INFRASTRUCTURE ONLY: imported by the tests and the CPU-baseline leg of
the benchmark; it never imports the product package.  Field arrays are
numpy complex128 [2 modes, 3 components (z, r, th), nr, nz] (z fastest);
particles are Cartesian positions and momenta [3, np] as (x, y, z) with z
the propagation axis (c = 1, lengths c/w_p).

The loading of the cylindrical plasma (random z and r in each (z, r) cell,
uniform azimuth, weight proportional to r so that the 3D density is the
profile's) is written here from its definition; the caller passes the
uniform random numbers in (a function of the counter array, the tests give
the seeded SplitMix64 stream they share with the GPU run).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import oracle as _O

_dp = ctypes.POINTER(ctypes.c_double)


class CircGrid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int64), ("nr", ctypes.c_int64), ("dz", ctypes.c_double), ("dr", ctypes.c_double),
                ("dt", ctypes.c_double)]


class CircLaser(ctypes.Structure):
    _fields_ = [("a0", ctypes.c_double), ("omega0", ctypes.c_double), ("waist", ctypes.c_double),
                ("fwhm", ctypes.c_double), ("t_peak", ctypes.c_double), ("t_end", ctypes.c_double),
                ("src", ctypes.c_int64)]


_ready = False


def lib():
    global _ready
    L = _O.lib()
    if not _ready:
        G, LP = ctypes.POINTER(CircGrid), ctypes.POINTER(CircLaser)
        i64, dbl = ctypes.c_int64, ctypes.c_double
        sig = {
            "circ_volume": (dbl, [G, i64]),
            "circ_shape_r": (None, [dbl, dbl, ctypes.POINTER(i64), _dp]),
            "circ_gather": (None, [G, _dp, _dp, _dp, _dp, _dp]),
            "circ_push": (ctypes.c_int, [G, i64, _dp, _dp, _dp, dbl, dbl, _dp, _dp]),
            "circ_deposit": (None, [G, i64, _dp, _dp, _dp, _dp, dbl, _dp]),
            "circ_rho": (None, [G, i64, _dp, _dp, dbl, _dp]),
            "circ_div": (None, [G, _dp, _dp]),
            "circ_field_step": (None, [G, _dp, _dp, _dp, LP, dbl]),
            "circ_window_shift": (None, [G, _dp, _dp]),
            "circ_field_energy": (dbl, [G, _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _ready = True
    return L


def _p(a):
    assert a.flags["C_CONTIGUOUS"] and a.dtype in (np.float64, np.complex128)
    return a.ctypes.data_as(_dp)


def make_grid(nz, nr, dz, dr, dt) -> CircGrid:
    return CircGrid(int(nz), int(nr), float(dz), float(dr), float(dt))


def make_laser(a0, omega0, waist, fwhm, t_peak, t_end, src) -> CircLaser:
    return CircLaser(float(a0), float(omega0), float(waist), float(fwhm), float(t_peak), float(t_end), int(src))


def zeros_field(g: CircGrid) -> np.ndarray:
    return np.zeros((2, 3, int(g.nr), int(g.nz)), dtype=np.complex128)


def volume(g, j) -> float:
    return lib().circ_volume(ctypes.byref(g), int(j))


def shape_r(r, dr):
    K = ctypes.c_int64()
    w = np.zeros(2)
    lib().circ_shape_r(float(r), float(dr), ctypes.byref(K), _p(w))
    return K.value, w


def gather(g, E, B, x):
    ep, bp = np.zeros(3), np.zeros(3)
    lib().circ_gather(ctypes.byref(g), _p(E), _p(B), _p(np.ascontiguousarray(x, dtype=np.float64)), _p(ep), _p(bp))
    return ep, bp


def push(g, x, u, E, B, q=-1.0, m=1.0):
    """Gather + Boris + move: returns (u_new, x_new)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    xn = np.zeros_like(x)
    st = lib().circ_push(ctypes.byref(g), x.shape[1], _p(x), _p(u), _p(xn), q, m, _p(E), _p(B))
    if st != 0:
        raise FloatingPointError("cylindrical oracle push produced a non-finite value")
    return u, xn


def deposit(g, x0, x1, u, w, q=-1.0):
    J = zeros_field(g)
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    x1 = np.ascontiguousarray(x1, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    lib().circ_deposit(ctypes.byref(g), x0.shape[1], _p(x0), _p(x1), _p(u), _p(w), q, _p(J))
    return J


def rho(g, x, w, q=-1.0):
    out = np.zeros((2, int(g.nr), int(g.nz)), dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.float64)
    lib().circ_rho(ctypes.byref(g), x.shape[1], _p(x), _p(np.ascontiguousarray(w, dtype=np.float64)), q, _p(out))
    return out


def div(g, F):
    out = np.zeros((2, int(g.nr), int(g.nz)), dtype=np.complex128)
    lib().circ_div(ctypes.byref(g), _p(np.ascontiguousarray(F)), _p(out))
    return out


def field_step(g, E, B, J=None, L=None, t=0.0):
    E, B = E.copy(), B.copy()
    Jp = _p(np.ascontiguousarray(J)) if J is not None else None
    lib().circ_field_step(ctypes.byref(g), _p(E), _p(B), Jp, ctypes.byref(L) if L is not None else None, float(t))
    return E, B


def window_shift(g, E, B):
    E, B = E.copy(), B.copy()
    lib().circ_window_shift(ctypes.byref(g), _p(E), _p(B))
    return E, B


def field_energy(g, E, B) -> float:
    return lib().circ_field_energy(ctypes.byref(g), _p(E), _p(B))


# ---------------------------------------------------------------- plasma loading

def density(z_lab, z_start, ramp, n_plateau):
    """Density profile along z (lab frame, c/w_p): 0 before z_start, linear
    over `ramp`, then n_plateau."""
    z = np.asarray(z_lab, dtype=np.float64)
    n = np.where(z < z_start, 0.0, np.where(z < z_start + ramp, n_plateau * (z - z_start) / max(ramp, 1e-300),
                                               n_plateau))
    return n


def load(g, plasma, shift, zb, ze, uniform, r_cells):
    """Cylindrical plasma of window z cells [zb, ze) after `shift` cells of
    window motion, radial cells [0, r_cells): ppc particles per (z, r) cell.

    Particle (lab cell Z, radial cell j, slot s) uses draws 3c, 3c+1, 3c+2 of
    `uniform` (counters -> uniforms in [0, 1)) with c = (Z nr + j) ppc + s:
    the z offset (rounded toward
    zero onto the 2^-24 lattice), the r offset and the azimuth / 2 pi.
    Position: z = (Z - shift + oz) dz in the window, r = (j + u_r) dr,
    (x, y) = r (cos th, sin th) rounded to FP32; weight
    n(z_lab) 2 pi r dr dz / ppc (FP32); none where n = 0.  Tag c mod 2^31.
    Returns dict(cell_z, oz, x (FP64 [3, np] from the FP32 values), w, id, u)."""
    ppc = int(plasma["ppc"])
    nr = int(g.nr)
    Z = np.arange(zb, ze, dtype=np.int64) + int(shift)
    Zg, jg, sg = np.meshgrid(Z, np.arange(r_cells, dtype=np.int64), np.arange(ppc, dtype=np.int64), indexing="ij")
    Zg, jg, sg = Zg.ravel(), jg.ravel(), sg.ravel()
    c = ((Zg * nr + jg) * ppc + sg).astype(np.uint64)
    uz = uniform(c * np.uint64(3))
    ur = uniform(c * np.uint64(3) + np.uint64(1))
    ut = uniform(c * np.uint64(3) + np.uint64(2))
    oz = (np.floor(uz * 2.0 ** 24) * 2.0 ** -24).astype(np.float32)    # toward zero onto the FP32 lattice
    r = (jg + ur) * g.dr
    th = 2.0 * math.pi * ut
    x = (r * np.cos(th)).astype(np.float32)
    y = (r * np.sin(th)).astype(np.float32)
    zl = (Zg + oz.astype(np.float64)) * g.dz
    n = density(zl, plasma["z_start"], plasma["ramp"], plasma["n_plateau"])
    keep = n > 0
    w = (n * 2.0 * math.pi * r * g.dr * g.dz / ppc).astype(np.float32)
    cz = (Zg - int(shift)).astype(np.int32)
    ids = (c.astype(np.int64) & 0x7FFFFFFF).astype(np.int32)
    X = np.stack([x.astype(np.float64), y.astype(np.float64), (cz + oz.astype(np.float64)) * g.dz])
    return {"cz": cz[keep], "oz": oz[keep], "x32": x[keep], "y32": y[keep], "x": X[:, keep], "w": w[keep],
            "id": ids[keep]}


def run(g, plasma, L, nsteps, window_start, period, uniform, r_cells, kill=2, wall=2, q=-1.0, m=1.0):
    """Moving-window quasi-cylindrical run in window coordinates.

    Start: vacuum fields, plasma of window z cells [0, nz - kill) and radial
    cells [0, r_cells).  Each step: push, deposit, field step with the laser
    source while the window has not moved and t <= t_end; then, after step
    n with n + 1 >= window_start and (n + 1 - window_start) % period == 0,
    the window moves one cell (fields shift, particles z -= dz, the plasma
    of the newly covered lab cell is loaded at window cell nz - 1 - kill).
    After every step particles outside window z cells [kill, nz - 1 - kill]
    or at r >= (nr - wall) dr are removed.
    Returns dict(x, u, w, id, E, B, J, shift)."""
    nz, nr = int(g.nz), int(g.nr)
    P = load(g, plasma, 0, 0, nz - kill, uniform, r_cells)
    x, w, ids = P["x"], P["w"].astype(np.float64), P["id"]
    u = np.zeros_like(x)
    E, B = zeros_field(g), zeros_field(g)
    J = zeros_field(g)
    shift = 0
    for n in range(nsteps):
        t = n * g.dt
        u, x1 = push(g, x, u, E, B, q, m)
        J = deposit(g, x, x1, u, w, q)
        E, B = field_step(g, E, B, J, L if (shift == 0 and L is not None and t <= L.t_end) else None, t)
        x = x1
        if n + 1 >= window_start and (n + 1 - window_start) % period == 0:
            E, B = window_shift(g, E, B)
            shift += 1
            x = x.copy()
            x[2] -= g.dz
            Q = load(g, plasma, shift, nz - 1 - kill, nz - kill, uniform, r_cells)
            x = np.concatenate([x, Q["x"]], axis=1)
            u = np.concatenate([u, np.zeros_like(Q["x"])], axis=1)
            w = np.concatenate([w, Q["w"].astype(np.float64)])
            ids = np.concatenate([ids, Q["id"]])
        r = np.sqrt(x[0] ** 2 + x[1] ** 2)
        keep = (x[2] >= kill * g.dz) & (x[2] < (nz - kill) * g.dz) & (r < (nr - wall) * g.dr)
        x, u, w, ids = x[:, keep], u[:, keep], w[keep], ids[keep]
    return {"x": x, "u": u, "w": w, "id": ids, "E": E, "B": B, "J": J, "shift": shift}
