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
_SRCS = (_SRC, os.path.join(_HERE, "denoise.c"), os.path.join(_HERE, "circ.c"))
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


class OraGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64 * 3), ("d", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("xbc", ctypes.c_int32), ("yzbc", ctypes.c_int32),
                ("alpha", ctypes.c_double * 3), ("beta", ctypes.c_double * 3), ("gam", ctypes.c_double * 3)]


def build(force: bool = False) -> str:
    """Compile oracle.c and denoise.c into liboracle.so with gcc (strict IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", *_SRCS, "-o", tmp, "-lm"])
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
            "ora_bf16": (dbl, [dbl]),
            "ora_conv3d": (None, [_i64p, _i32p, i64, _dp, i32, _dp, _dp, i32, _dp]),
            "ora_denoise": (i32, [_i64p, _i32p, i64, _dp, _dp, _dp, i32, _dp, _dp, _dp, _dp, _dp, _dp, i32, _dp,
                                  _dp]),
            "ora_denoise_grad": (dbl, [_i64p, _i32p, i64, _dp, _dp, _dp, _dp, _dp, i32, _dp, _dp, _dp, _dp, _dp, _dp,
                                       _dp, _dp, _dp, _dp, _dp, _dp]),
            "ora_denoise_sigma": (dbl, [_dp, _dp]),
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


def make_grid(n, d, dt, solver: str = "yee", xbc: int = 0, variant: int = 0, coeffs=None, yzbc: int = 0) -> OraGrid:
    g = OraGrid()
    g.yzbc = int(yzbc)
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


class OraLaser(ctypes.Structure):
    _fields_ = [("a0", ctypes.c_double), ("omega0", ctypes.c_double), ("waist", ctypes.c_double),
                ("fwhm", ctypes.c_double), ("t_peak", ctypes.c_double), ("t_end", ctypes.c_double),
                ("yc", ctypes.c_double), ("zc", ctypes.c_double), ("src_x", ctypes.c_int64)]


class OraPlasma(ctypes.Structure):
    _fields_ = [("x_start", ctypes.c_double), ("ramp", ctypes.c_double), ("n_plateau", ctypes.c_double),
                ("ppc", ctypes.c_int32 * 3)]


def _lwfa_sigs():
    L = lib()
    G, LP, PP = ctypes.POINTER(OraGrid), ctypes.POINTER(OraLaser), ctypes.POINTER(OraPlasma)
    i64, dbl = ctypes.c_int64, ctypes.c_double
    sig = {
        "ora_laser_e": (dbl, [LP, dbl]),
        "ora_laser_profile": (dbl, [LP, dbl, dbl]),
        "ora_field_step_laser": (None, [G, _dp, _dp, _dp, LP, dbl]),
        "ora_window_shift": (None, [G, _dp, _dp]),
        "ora_density": (dbl, [PP, dbl]),
        "ora_inject": (i64, [G, PP, i64, i64, i64, _dp, _dp, ctypes.POINTER(ctypes.c_int32), i64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def make_laser(a0, omega0, waist, fwhm, t_peak, t_end, yc, zc, src_x) -> OraLaser:
    return OraLaser(float(a0), float(omega0), float(waist), float(fwhm), float(t_peak), float(t_end), float(yc),
                    float(zc), int(src_x))


def make_plasma(x_start, ramp, n_plateau, ppc=(2, 2, 2)) -> OraPlasma:
    p = OraPlasma(float(x_start), float(ramp), float(n_plateau))
    for a in range(3):
        p.ppc[a] = int(ppc[a])
    return p


def laser_e(L: OraLaser, t: float) -> float:
    return _lwfa_sigs().ora_laser_e(ctypes.byref(L), float(t))


def laser_profile(L: OraLaser, y: float, z: float) -> float:
    return _lwfa_sigs().ora_laser_profile(ctypes.byref(L), float(y), float(z))


def density(P: OraPlasma, x_cells: float) -> float:
    return _lwfa_sigs().ora_density(ctypes.byref(P), float(x_cells))


def field_step_laser(g: OraGrid, E, B, J, L: OraLaser, t: float):
    E, B = f64(E).copy(), f64(B).copy()
    Jp = _p(f64(J)) if J is not None else None
    Lp = ctypes.byref(L) if L is not None else None
    _lwfa_sigs().ora_field_step_laser(ctypes.byref(g), _p(E), _p(B), Jp, Lp, float(t))
    return E, B


def window_shift(g: OraGrid, E, B):
    E, B = f64(E).copy(), f64(B).copy()
    _lwfa_sigs().ora_window_shift(ctypes.byref(g), _p(E), _p(B))
    return E, B


def inject(g: OraGrid, P: OraPlasma, shift: int, xb: int, xe: int):
    """Cold lattice plasma of window cells [xb, xe): (x[3, m] window positions, w[m], id[m])."""
    ppc = P.ppc[0] * P.ppc[1] * P.ppc[2]
    cap = max(1, (xe - xb) * int(g.n[1]) * int(g.n[2]) * ppc)
    x = np.zeros((3, cap))
    w = np.zeros(cap)
    ids = np.zeros(cap, dtype=np.int32)
    m = _lwfa_sigs().ora_inject(ctypes.byref(g), ctypes.byref(P), int(shift), int(xb), int(xe), _p(x), _p(w),
                                ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    return x[:, :m].copy(), w[:m].copy(), ids[:m].copy()


def run_lwfa(g: OraGrid, P: OraPlasma, L: OraLaser, nsteps: int, window_start: int, kill_lo: int = 3,
             inject_hi: int = 3, jpost: int = 0, q=-1.0, m=1.0, pml=None):
    """Moving-window laser-wakefield run in window coordinates (c = 1, c dt = dx).

    Start: vacuum fields, plasma loaded over window cells [0, nx - inject_hi).
    Each step: push, deposit, optional binomial filter, field step with the
    laser source while the window has not moved; then, from step
    `window_start` on, the window moves one cell (fields shift, the leading
    plane is cleared and the plasma of the newly covered lab cell is loaded
    at window cell nx - 1 - inject_hi).  After every step particles outside
    window cells [kill_lo, nx - 1 - inject_hi] are removed (their shapes
    would reach past the window's ends).

    pml (an OraPml, grid with both yzbc bits): the transverse layer in the
    field update, its auxiliary arrays moving with the window, and particles
    whose transverse cell lies in the layer are removed with the others
    (also right after loading, i.e. before they ever move).
    Returns dict(x, u, w, id, E, B, J, shift).
    """
    nx = int(g.n[0])
    x, w, ids = inject(g, P, 0, 0, nx - inject_hi)
    u = np.zeros_like(x)
    E = zeros_field(g)
    B = zeros_field(g)
    psi = zeros_psi(g) if pml is not None else None
    shift = 0
    J = zeros_field(g)

    def kept(x):
        k = (x[0] >= kill_lo * g.d[0]) & (x[0] < (nx - inject_hi) * g.d[0])
        if pml is not None:
            lay = int(pml.layers)
            for a in (1, 2):
                c = np.floor(x[a] / g.d[a])
                k &= (c >= lay) & (c < int(g.n[a]) - lay)
        return k

    if pml is not None:
        keep = kept(x)
        x, u, w, ids = x[:, keep], u[:, keep], w[keep], ids[keep]
    for n in range(nsteps):
        t = n * g.dt
        x0 = x.copy()
        xw, u, x1 = push(g, x, u, E, B, q, m)
        J = deposit(g, x0, x1, w, q)
        if jpost == 1:
            J = binomial(g, J)
        Ln = L if (shift == 0 and t <= L.t_end) else None
        if pml is not None:
            E, B, psi = field_step_laser_pml(g, E, B, J, Ln, t, pml, psi)
        else:
            E, B = field_step_laser(g, E, B, J, Ln, t)
        x = xw
        if n + 1 >= window_start:
            E, B = window_shift(g, E, B)
            if pml is not None:
                psi = pml_window_shift(g, psi)
            shift += 1
            x[0] -= g.d[0]
            xn, wn, idn = inject(g, P, shift, nx - 1 - inject_hi, nx - inject_hi)
            x = np.concatenate([x, xn], axis=1)
            u = np.concatenate([u, np.zeros_like(xn)], axis=1)
            w = np.concatenate([w, wn])
            ids = np.concatenate([ids, idn])
        keep = kept(x)
        x, u, w, ids = x[:, keep], u[:, keep], w[keep], ids[keep]
    return {"x": x, "u": u, "w": w, "id": ids, "E": E, "B": B, "J": J, "shift": shift, "psi": psi}


class OraPml(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int64), ("sigma_max", ctypes.c_double * 3), ("grade", ctypes.c_double)]


def make_pml(g: OraGrid, layers: int = 16, sigma_max=None, grade: float = 3.0, axes=(1, 2)) -> OraPml:
    """Transverse layer of `layers` cells on the given axes; sigma_max per
    axis (default 0.8 (grade + 1) / d), profile sigma_max depth^grade."""
    P = OraPml()
    P.layers = int(layers)
    P.grade = float(grade)
    for a in axes:
        P.sigma_max[a] = float(sigma_max if sigma_max is not None else 0.8 * (grade + 1.0) / g.d[a])
    return P


def _pml_sigs():
    L = lib()
    G, PP, LP = ctypes.POINTER(OraGrid), ctypes.POINTER(OraPml), ctypes.POINTER(OraLaser)
    for name, (res, args) in {"ora_pml_field_step": (None, [G, PP, _dp, _dp, _dp, _dp]),
                              "ora_pml_sigma": (ctypes.c_double, [PP, ctypes.c_int, ctypes.c_int64, ctypes.c_double]),
                              "ora_field_step_laser_pml": (None, [G, _dp, _dp, _dp, LP, ctypes.c_double, PP, _dp]),
                              "ora_pml_window_shift": (None, [G, _dp]),
                              }.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    return L


def zeros_psi(g: OraGrid) -> np.ndarray:
    return np.zeros((8,) + _fshape(g)[1:])


def pml_field_step(g: OraGrid, P: OraPml, E, B, psi, J=None):
    """One field step with the transverse layer; returns (E, B, psi) (copies)."""
    E, B, psi = f64(E).copy(), f64(B).copy(), f64(psi).copy()
    Jp = _p(f64(J)) if J is not None else None
    _pml_sigs().ora_pml_field_step(ctypes.byref(g), ctypes.byref(P), _p(E), _p(B), Jp, _p(psi))
    return E, B, psi


def pml_sigma(P: OraPml, axis: int, n: int, p: float) -> float:
    return _pml_sigs().ora_pml_sigma(ctypes.byref(P), int(axis), int(n), float(p))


def field_step_laser_pml(g: OraGrid, E, B, J, L, t: float, P: OraPml, psi):
    """field_step_laser with the transverse layer; returns (E, B, psi) (copies)."""
    E, B, psi = f64(E).copy(), f64(B).copy(), f64(psi).copy()
    Jp = _p(f64(J)) if J is not None else None
    Lp = ctypes.byref(L) if L is not None else None
    _pml_sigs().ora_field_step_laser_pml(ctypes.byref(g), _p(E), _p(B), Jp, Lp, float(t), ctypes.byref(P), _p(psi))
    return E, B, psi


def pml_window_shift(g: OraGrid, psi):
    psi = f64(psi).copy()
    _pml_sigs().ora_pml_window_shift(ctypes.byref(g), _p(psi))
    return psi


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


# ---------------------------------------------------------------- current denoiser (denoise.c)

BC = {"periodic": 0, "zero": 1, "window": 2}


def bf16(x: float) -> float:
    """Nearest bfloat16 value (ties to even)."""
    return lib().ora_bf16(float(x))


def _dims(n, bc):
    nn = (ctypes.c_int64 * 3)(*[int(v) for v in n])
    b = (ctypes.c_int32 * 3)(*[BC[v] if isinstance(v, str) else int(v) for v in bc])
    return nn, b


def conv3d(inp, W, b=None, bc=("periodic",) * 3, origin: int = 0):
    """3x3x3 cross-correlation: inp [cin, nz, ny, nx], W [cout, cin, 3, 3, 3] ([z][y][x] taps)."""
    inp = f64(inp)
    W = f64(W)
    cin, nz, ny, nx = inp.shape
    cout = W.shape[0]
    assert W.shape == (cout, cin, 3, 3, 3)
    out = np.zeros((cout, nz, ny, nx))
    nn, bb = _dims((nx, ny, nz), bc)
    bias = f64(b) if b is not None else None
    lib().ora_conv3d(nn, bb, int(origin), _p(inp), cin, _p(W), _p(bias) if bias is not None else None, cout,
                     _p(out))
    return out


def denoise(J, scale, params, d=(1.0, 1.0, 1.0), bc=("periodic",) * 3, origin: int = 0, round_bf16: bool = True):
    """(Jout, y) of the denoiser; J [3, nz, ny, nx]; params = (W1, b1, W2, b2, W3, b3); d = cell sizes."""
    J = f64(J)
    _, nz, ny, nx = J.shape
    W1, b1, W2, b2, W3, b3 = [f64(a) for a in params]
    H = W1.shape[0]
    Jout = np.zeros_like(J)
    y = np.zeros_like(J)
    nn, bb = _dims((nx, ny, nz), bc)
    sc = f64(scale)
    dd = f64(d)
    st = lib().ora_denoise(nn, bb, int(origin), _p(dd), _p(J), _p(sc), H, _p(W1), _p(b1), _p(W2), _p(b2), _p(W3),
                           _p(b3), 1 if round_bf16 else 0, _p(Jout), _p(y))
    if st != 0:
        raise MemoryError("oracle denoiser")
    return Jout, y


def denoise_sigma(d, scale) -> float:
    return lib().ora_denoise_sigma(_p(f64(d)), _p(f64(scale)))


def denoise_grad(J, x, T, scale, params, d=(1.0, 1.0, 1.0), bc=("zero",) * 3, origin: int = 0):
    """(loss, grads) of the training loss mean(((Jout - T) / s)^2); x is the network input (bf16(J/s))."""
    J = f64(J)
    x = f64(x)
    T = f64(T)
    _, nz, ny, nx = J.shape
    P = [f64(a) for a in params]
    G = [np.zeros_like(a) for a in P]
    H = P[0].shape[0]
    nn, bb = _dims((nx, ny, nz), bc)
    loss = lib().ora_denoise_grad(nn, bb, int(origin), _p(f64(d)), _p(J), _p(x), _p(T), _p(f64(scale)), H,
                                  *[_p(a) for a in P], *[_p(g) for g in G])
    return loss, G
