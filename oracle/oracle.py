"""Python access to the FP64 reference PIC cycle in ``oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  It shares no code with the HIP library
and never imports the product package.  Arrays are numpy float64:
fields ``[3, nz, ny, nx]`` (component-major, x fastest), particle positions
and momenta ``[3, np]`` in plasma-normalised units (c = eps0 = 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


class OraGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64 * 3), ("d", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("xbc", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("alpha", ctypes.c_double * 3), ("beta", ctypes.c_double * 3), ("gam", ctypes.c_double * 3)]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (strict IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        G = ctypes.POINTER(OraGrid)
        i64, dbl, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        sig = {
            "ora_bspline3": (dbl, [dbl]),
            "ora_gather": (None, [G, _dp, _dp, _dp, _dp, _dp]),
            "ora_boris": (None, [_dp, _dp, _dp, dbl, dbl]),
            "ora_push": (i32, [G, i64, _dp, _dp, _dp, dbl, dbl, _dp, _dp]),
            "ora_deposit": (None, [G, i64, _dp, _dp, _dp, dbl, _dp]),
            "ora_rho": (None, [G, i64, _dp, _dp, dbl, _dp]),
            "ora_continuity": (dbl, [G, _dp, _dp, _dp, _dp]),
            "ora_field_step": (None, [G, _dp, _dp, _dp]),
            "ora_b_half": (None, [G, _dp, _dp, dbl]),
            "ora_div_e": (None, [G, _dp, _dp]),
            "ora_div_b": (None, [G, _dp, _dp]),
            "ora_binomial": (None, [G, _dp]),
            "ora_pd_coeffs": (i32, [_dp, i32, _dp, _dp, _dp]),
            "ora_diag": (None, [G, i64, _dp, _dp, dbl, dbl, _dp, _dp, _dp, _dp]),
            "ora_step": (i32, [G, i64, _dp, _dp, _dp, dbl, dbl, _dp, _dp, _dp, i32, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous float64"
    return a.ctypes.data_as(_dp)


def f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def pd_coeffs(d, variant: int = 0):
    """(alpha, beta, gamma) of the smoothing stencils; variant 0 = with corners,
    1 = no corners, 2 = identity (Yee)."""
    a, b, g = (np.zeros(3) for _ in range(3))
    st = lib().ora_pd_coeffs(_p(f64(d)), variant, _p(a), _p(b), _p(g))
    if st != 0:
        raise ValueError("perfect dispersion needs dx <= dy, dz")
    return a, b, g


def make_grid(n, d, dt, solver: str = "yee", xbc: int = 0, variant: int = 0, coeffs=None) -> OraGrid:
    g = OraGrid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.d[a] = float(d[a])
    g.dt = float(dt)
    g.xbc = int(xbc)
    if coeffs is None:
        coeffs = pd_coeffs(d, 2 if solver == "yee" else variant)
    for a in range(3):
        g.alpha[a], g.beta[a], g.gam[a] = coeffs[0][a], coeffs[1][a], coeffs[2][a]
    return g


def from_grid(grid, variant: int = 0) -> OraGrid:
    """OraGrid from an ``inputs.Grid``-like object (n, d, dt, solver, window)."""
    return make_grid(grid.n, grid.d, grid.dt, grid.solver, 1 if getattr(grid, "window", False) else 0, variant)


def _ncell(g: OraGrid) -> int:
    return int(g.n[0] * g.n[1] * g.n[2])


def _fshape(g: OraGrid):
    return (3, int(g.n[2]), int(g.n[1]), int(g.n[0]))


def zeros_field(g: OraGrid) -> np.ndarray:
    return np.zeros(_fshape(g))


def bspline3(xi: float) -> float:
    return lib().ora_bspline3(float(xi))


def gather(g: OraGrid, E, B, x):
    E, B, x = f64(E), f64(B), f64(x)
    ep, bp = np.zeros(3), np.zeros(3)
    lib().ora_gather(ctypes.byref(g), _p(E), _p(B), _p(x), _p(ep), _p(bp))
    return ep, bp


def boris(u, E, B, qm: float, dt: float):
    u = f64(u).copy()
    lib().ora_boris(_p(u), _p(f64(E)), _p(f64(B)), qm, dt)
    return u


def push(g: OraGrid, x, u, E, B, q=-1.0, m=1.0):
    """Gather + Boris + move.  Returns (x_wrapped, u_new, x_unwrapped)."""
    x, u = f64(x).copy(), f64(u).copy()
    np_ = x.shape[1]
    xn = np.zeros_like(x)
    st = lib().ora_push(ctypes.byref(g), np_, _p(x), _p(u), _p(xn), q, m, _p(f64(E)), _p(f64(B)))
    if st != 0:
        raise FloatingPointError("oracle push produced a non-finite value")
    return x, u, xn


def deposit(g: OraGrid, x0, x1, w, q=-1.0, J=None):
    x0, x1, w = f64(x0), f64(x1), f64(w)
    J = zeros_field(g) if J is None else f64(J).copy()
    lib().ora_deposit(ctypes.byref(g), x0.shape[1], _p(x0), _p(x1), _p(w), q, _p(J))
    return J


def rho(g: OraGrid, x, w, q=-1.0):
    x, w = f64(x), f64(w)
    r = np.zeros(_fshape(g)[1:])
    lib().ora_rho(ctypes.byref(g), x.shape[1], _p(x), _p(w), q, _p(r))
    return r


def continuity(g: OraGrid, rho0, rho1, J):
    res = np.zeros(_fshape(g)[1:])
    mx = lib().ora_continuity(ctypes.byref(g), _p(f64(rho0)), _p(f64(rho1)), _p(f64(J)), _p(res))
    return mx, res


def field_step(g: OraGrid, E, B, J=None):
    E, B = f64(E).copy(), f64(B).copy()
    Jp = _p(f64(J)) if J is not None else None
    lib().ora_field_step(ctypes.byref(g), _p(E), _p(B), Jp)
    return E, B


def b_half(g: OraGrid, E, B, h: float):
    B = f64(B).copy()
    lib().ora_b_half(ctypes.byref(g), _p(f64(E)), _p(B), h)
    return B


def div_e(g: OraGrid, E):
    out = np.zeros(_fshape(g)[1:])
    lib().ora_div_e(ctypes.byref(g), _p(f64(E)), _p(out))
    return out


def div_b(g: OraGrid, B):
    out = np.zeros(_fshape(g)[1:])
    lib().ora_div_b(ctypes.byref(g), _p(f64(B)), _p(out))
    return out


def binomial(g: OraGrid, J):
    J = f64(J).copy()
    lib().ora_binomial(ctypes.byref(g), _p(J))
    return J


def diag(g: OraGrid, u, w, E, B, J=None, q=-1.0, m=1.0):
    u, w = f64(u), f64(w)
    out = np.zeros(4)
    Jp = _p(f64(J)) if J is not None else None
    lib().ora_diag(ctypes.byref(g), u.shape[1], _p(u), _p(w), q, m, _p(f64(E)), _p(f64(B)), Jp, _p(out))
    return {"charge": out[0], "e_field": out[1], "e_kin": out[2], "max_abs_J": out[3]}


def step(g: OraGrid, x, u, w, E, B, q=-1.0, m=1.0, jpost: int = 0):
    """One PIC step in place on copies.  Returns dict(x, u, E, B, J, x_prev)."""
    x, u, E, B, w = f64(x).copy(), f64(u).copy(), f64(E).copy(), f64(B).copy(), f64(w)
    np_ = x.shape[1]
    J = zeros_field(g)
    xp = np.zeros_like(x)
    st = lib().ora_step(ctypes.byref(g), np_, _p(x), _p(u), _p(w), q, m, _p(E), _p(B), _p(J), jpost, _p(xp))
    if st != 0:
        raise FloatingPointError("oracle step produced a non-finite value")
    return {"x": x, "u": u, "E": E, "B": B, "J": J, "x_prev": xp}
