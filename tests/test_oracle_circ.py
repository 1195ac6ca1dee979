"""Pins of the quasi-cylindrical (m = 0, 1) oracle (oracle/circ.c, circ.py).

- The radial shape is density-conserving: a uniform 3D density deposits
  exactly n V_j on every node, the axis node included (closed-form volumes,
  by quadrature of the oracle's shape).
- A field uniform across the axis (E_x = const, E_z = const, B_z = const)
  is gathered exactly at any position, near the axis too.
- A transversely uniform m = 1 wave (linear polarisation) evolves exactly as
  the 3D Cartesian oracle's plane wave on a grid with the same axial
  spacing: two independent field solvers, the axis rules included, agree
  to round-off away from the radial wall; so does the laser source.
- The m = 0 and m = 1 TM and TE cavity modes of a conducting cylinder
  (E_z = J_m(j_m1 r / R) cos(omega t), omega = j_m1 / R, or B_z with the
  zeros of J_m') converge at second order in the cell size.
- The deposit obeys each mode's discrete continuity equation to round-off
  (m = 0 on every node, m = 1 off the axis), and in whole PIC steps Gauss's
  law div E - rho stays constant.

Each pin also rejects copies of the oracle with a planted mistake.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest
from scipy import special

from oracle import circ as C
from oracle import oracle as O


def test_radial_shape_is_density_conserving():
    dr = 0.2
    nodes = 6
    # integral of 2 pi r S_j(r) over r, by a fine midpoint rule of the oracle's weights
    M = 4000
    acc = np.zeros(nodes + 1)
    for K in range(nodes):
        s = (np.arange(M) + 0.5) / M
        for si in s:
            r = (K + si) * dr
            k, w = C.shape_r(r, dr)
            assert k == K and abs(w.sum() - 1.0) < 1e-15 and w.min() >= 0.0
            acc[k] += 2 * math.pi * r * w[0] * dr / M
            acc[k + 1] += 2 * math.pi * r * w[1] * dr / M
    want = [math.pi * dr * dr / 4] + [2 * math.pi * j * dr * dr for j in range(1, nodes)]
    assert np.allclose(acc[:nodes], want, rtol=1e-6, atol=0)
    g = C.make_grid(8, 8, 0.05, dr, 0.02)
    for j in range(4):
        assert abs(C.volume(g, j) - want[j] * 0.05) < 1e-15
    # continuity of the weights across cell boundaries
    for K in range(1, nodes):
        k_lo, w_lo = C.shape_r(K * dr - 1e-12, dr)
        k_hi, w_hi = C.shape_r(K * dr, dr)
        assert abs(w_lo[1] - w_hi[0]) < 1e-9


def test_uniform_fields_are_gathered_exactly():
    g = C.make_grid(12, 10, 0.05, 0.2, 0.02)
    E, B = C.zeros_field(g), C.zeros_field(g)
    ex, ez, bz = 0.7, -0.3, 1.1
    E[1, 1] = ex                 # m = 1 E_r
    E[1, 2] = -1j * ex           # m = 1 E_th
    E[0, 0] = ez                 # m = 0 E_z
    B[0, 0] = bz                 # m = 0 B_z
    rng = np.random.default_rng(3)
    for _ in range(200):
        r = rng.uniform(0, 1.4) if rng.random() < 0.7 else rng.uniform(0, 0.15)
        th = rng.uniform(0, 2 * math.pi)
        x = np.array([r * math.cos(th), r * math.sin(th), rng.uniform(0.1, 0.45)])
        ep, bp = C.gather(g, E, B, x)
        assert np.allclose(ep, [ex, 0.0, ez], atol=1e-14) and np.allclose(bp, [0.0, 0.0, bz], atol=1e-14)


def _uniform_m1_wave(g, ey3, bz3):
    """m = 1 fields of E_x = ey3(z), B_y = bz3(z), uniform across the axis."""
    E, B = C.zeros_field(g), C.zeros_field(g)
    E[1, 1] = ey3[None, :]
    E[1, 2] = -1j * ey3[None, :]
    B[1, 2] = bz3[None, :]
    B[1, 1] = 1j * bz3[None, :]
    return E, B


def test_uniform_m1_wave_matches_the_cartesian_solver():
    nz, nr, dz, dr, dt = 96, 100, 0.05, 0.2, 0.03
    g = C.make_grid(nz, nr, dz, dr, dt)
    g3 = O.make_grid((nz, 4, 4), (dz, 0.5, 0.5), dt, solver="yee", xbc=1)
    xs = np.arange(nz) * dz
    ey = np.exp(-((xs - 2.4) / 0.4) ** 2) * np.cos(9.0 * xs)
    E3, B3 = O.zeros_field(g3), O.zeros_field(g3)
    E3[1] = ey[None, None, :]
    E, B = _uniform_m1_wave(g, ey, np.zeros(nz))
    steps = 40
    for _ in range(steps):
        E3, B3 = O.field_step(g3, E3, B3)
        E, B = C.field_step(g, E, B)
    inner = 60                 # the wall's zero E_th reaches ~15 cells in by the stencils' spread
    e3, b3 = E3[1, 0, 0, :], B3[2, 0, 0, :]
    assert np.abs(e3).max() > 0.3
    assert np.abs(E[1, 1, :inner] - e3[None, :]).max() < 1e-13
    assert np.abs(E[1, 2, :inner] + 1j * e3[None, :]).max() < 1e-13
    assert np.abs(B[1, 2, :inner] - b3[None, :]).max() < 1e-13
    assert np.abs(B[1, 1, :inner] - 1j * b3[None, :]).max() < 1e-13
    assert np.abs(E[1, 0]).max() < 1e-13 and np.abs(E[0]).max() == 0 and np.abs(B[0]).max() == 0


def test_uniform_m1_laser_source_matches_the_cartesian_source():
    nz, nr, dz, dr, dt = 120, 130, 0.05, 0.2, 0.025
    g = C.make_grid(nz, nr, dz, dr, dt)
    g3 = O.make_grid((nz, 4, 4), (dz, 0.5, 0.5), dt, solver="yee", xbc=1)
    L = C.make_laser(a0=0.5, omega0=8.0, waist=1e12, fwhm=0.6, t_peak=1.0, t_end=1.6, src=4)
    L3 = O.make_laser(a0=0.5, omega0=8.0, waist=1e12, fwhm=0.6, t_peak=1.0, t_end=1.6, yc=1.0, zc=1.0, src_x=4)
    E, B = C.zeros_field(g), C.zeros_field(g)
    E3, B3 = O.zeros_field(g3), O.zeros_field(g3)
    steps = 80
    for n in range(steps):
        t = n * dt
        E, B = C.field_step(g, E, B, None, L, t)
        E3, B3 = O.field_step_laser(g3, E3, B3, None, L3, t)
    inner = 60
    e3 = E3[1, 0, 0, :]
    assert np.abs(e3).max() > 0.5
    assert np.abs(E[1, 1, :inner] - e3[None, :]).max() < 1e-12 * np.abs(e3).max()
    assert np.abs(E[1, 2, :inner] + 1j * e3[None, :]).max() < 1e-12 * np.abs(e3).max()


def _jm_over_r(m, k, r):
    """J_m(k r) / r with its limit k/2 (m = 1) or 0 (m = 0) on the axis... times m."""
    out = np.zeros_like(r)
    nz = r > 0
    out[nz] = m * special.jv(m, k * r[nz]) / r[nz]
    if m == 1:
        out[~nz] = k / 2
    return out


def _cavity_error(m, nr, te=False):
    """Max error at t = 5/4 period of the TM_m10 mode (E_z = J_m(k r) cos(w t),
    k = j_m1 / R, B_r = (i m / r) J_m sin(w t) / w, B_th = k J_m' sin(w t) / w)
    or the TE_m10 mode (B_z = J_m(k r) cos(w t), k = j'_m1 / R,
    E_r = -(i m / r) J_m sin / w, E_th = -k J_m' sin / w) of a conducting
    cylinder of radius 1, uniform in z, against the Bessel solution at every
    stored node, the axis included (interior z only)."""
    R = 1.0
    dr = R / nr
    dz = dr
    jm1 = (special.jnp_zeros(m, 1) if te else special.jn_zeros(m, 1))[0]
    k = jm1 / R
    T = 2 * math.pi / k
    dt = 0.4 * dz
    steps = int(round(1.25 * T / dt))
    dt = 1.25 * T / steps
    nz = int(2 * (1.25 * T + 0.5) / dz) + 8
    g = C.make_grid(nz, nr, dz, dr, dt)
    E, B = C.zeros_field(g), C.zeros_field(g)
    ri = np.arange(nr) * dr                  # integer r nodes
    rh = (np.arange(nr) + 0.5) * dr          # half r nodes
    # the standing mode is cos(w t): the other field is zero at t = 0
    F = B if te else E
    F[m, 0] = special.jv(m, k * (rh if te else ri))[:, None] * np.ones(nz)[None, :]
    for _ in range(steps):
        E, B = C.field_step(g, E, B)
    t = steps * dt
    c, sn = math.cos(k * t), math.sin(k * t) / k
    mid = slice(nz // 2 - 2, nz // 2 + 2)
    if te:
        pairs = [(B[m, 0], special.jv(m, k * rh) * c),
                 (E[m, 1], -1j * _jm_over_r(m, k, rh) * sn),
                 (E[m, 2], -k * special.jvp(m, k * ri) * sn)]
    else:
        pairs = [(E[m, 0], special.jv(m, k * ri) * c),
                 (B[m, 1], 1j * _jm_over_r(m, k, ri) * sn),
                 (B[m, 2], k * special.jvp(m, k * rh) * sn)]
    return max(np.abs(got[:, mid] - want[:, None]).max() for got, want in pairs)


@pytest.mark.parametrize("m,te", [(0, False), (1, False), (0, True), (1, True)])
def test_cavity_modes_converge_at_second_order(m, te):
    e1, e2 = _cavity_error(m, 12, te), _cavity_error(m, 24, te)
    assert e1 < 0.04, e1              # 0.003-0.03 at 12 cells per radius
    assert e1 / e2 > 3.2, (e1, e2)   # 3.3-4.0 measured


def _random_moves(g, n, seed, near_axis=False):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.0, 0.5, n) if near_axis else rng.uniform(0.0, (int(g.nr) - 4) * g.dr, n)
    th = rng.uniform(0, 2 * math.pi, n)
    z = rng.uniform(4 * g.dz, (int(g.nz) - 4) * g.dz, n)
    x0 = np.stack([r * np.cos(th), r * np.sin(th), z])
    step = rng.uniform(-1, 1, (3, n)) * np.array([[0.6 * g.dr], [0.6 * g.dr], [0.9 * g.dz]])
    x1 = x0 + step
    u = rng.normal(0, 0.5, (3, n))
    w = rng.uniform(0.5, 1.5, n)
    return x0, x1, u, w


@pytest.mark.parametrize("near_axis", [False, True])
def test_deposit_obeys_each_modes_continuity_equation(near_axis):
    g = C.make_grid(24, 12, 0.05, 0.2, 0.04)
    x0, x1, u, w = _random_moves(g, 400, 5 + near_axis, near_axis)
    J = C.deposit(g, x0, x1, u, w)
    r0, r1 = C.rho(g, x0, w), C.rho(g, x1, w)
    res = (r1 - r0) / g.dt + C.div(g, J)
    jmax = np.abs(J).max()
    assert jmax > 0
    assert np.abs(res[0]).max() < 1e-12 * jmax / g.dr
    assert np.abs(res[1, 1:]).max() < 1e-12 * jmax / g.dr
    # the charge itself: the m = 0 density integrates to the particles' charge
    vol = np.array([C.volume(g, j) for j in range(int(g.nr))])
    assert abs((r0[0].real * vol[:, None]).sum() + w.sum()) < 1e-12 * w.sum()


def test_gauss_law_is_kept_through_pic_steps():
    g = C.make_grid(24, 12, 0.05, 0.2, 0.02)
    rng = np.random.default_rng(9)
    n = 300
    r = rng.uniform(0.0, 1.2, n)
    th = rng.uniform(0, 2 * math.pi, n)
    x = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(0.4, 0.8, n)])
    u = rng.normal(0, 0.3, (3, n))
    w = rng.uniform(0.5, 1.5, n)
    E, B = C.zeros_field(g), C.zeros_field(g)
    gauss0 = C.div(g, E) - C.rho(g, x, w)
    for _ in range(12):
        u, x1 = C.push(g, x, u, E, B)
        J = C.deposit(g, x, x1, u, w)
        E, B = C.field_step(g, E, B, J)
        x = x1
    gauss = C.div(g, E) - C.rho(g, x, w)
    scale = np.abs(gauss0).max()
    assert np.abs(E).max() > 1e-3
    assert np.abs(gauss[0] - gauss0[0]).max() < 1e-11 * scale
    assert np.abs(gauss[1, 1:] - gauss0[1, 1:]).max() < 1e-11 * scale


# ---------------------------------------------------------------- planted mistakes
MUTANTS = [
    ("axis_flux_factor", "tz[f] = m == 0 ? 4.0 * at(g, Bt, i, 0) / g->dr : 0.0;",
     "tz[f] = m == 0 ? 2.0 * at(g, Bt, i, 0) / g->dr : 0.0;", lambda: test_cavity_modes_converge_at_second_order(0, False)),
    ("axis_dr_bz_factor", "- 2.0 * at(g, Bz, i, 0) / g->dr;", "- 1.0 * at(g, Bz, i, 0) / g->dr;",
     lambda: test_cavity_modes_converge_at_second_order(1, True)),
    ("plain_linear_radial_shape", "double f = s + s * (1.0 - s) / (2.0 * (2.0 * (double)k + 1.0));",
     "double f = s;", test_radial_shape_is_density_conserving),
    ("esirkepov_third_dropped", "+ 0.5 * a0[ii] * db[jj] +\n                                    da[ii] * db[jj] / 3.0);",
     "+ 0.5 * a0[ii] * db[jj]);", lambda: test_deposit_obeys_each_modes_continuity_equation(False)),
    ("jtheta_sign", "add(g, J, 1, 2, bz + ii, j, -I * rj", "add(g, J, 1, 2, bz + ii, j, I * rj",
     lambda: test_deposit_obeys_each_modes_continuity_equation(False)),
    ("er_ghost_parity", "else if (c == 1) v = interp_half(g, C, z, r, 0.0, m == 1 ? 1.0 : -1.0);",
     "else if (c == 1) v = interp_half(g, C, z, r, 0.0, m == 1 ? -1.0 : 1.0);", test_uniform_fields_are_gathered_exactly),
    ("m1_br_axis", "-I * at(g, Ez, i, 1) / g->dr - (at(g, Et, i + 1, 0) - at(g, Et, i, 0)) / g->dz;",
     "- (at(g, Et, i + 1, 0) - at(g, Et, i, 0)) / g->dz;", lambda: test_cavity_modes_converge_at_second_order(1, False)),
    ("laser_br_sign", "B[(1 * 3 + 1) * N + j * g->nz + i] += I * h * e * fj / g->dz;",
     "B[(1 * 3 + 1) * N + j * g->nz + i] -= I * h * e * fj / g->dz;", test_uniform_m1_laser_source_matches_the_cartesian_source),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_rejects_planted_mistake(tmp_path, monkeypatch, name, old, new, pin):
    import shutil

    d = tmp_path / name
    d.mkdir()
    src_dir = os.path.dirname(O.__file__)
    for f in ("oracle.c", "denoise.c", "circ.c"):
        shutil.copy(os.path.join(src_dir, f), d / f)
    text = (d / "circ.c").read_text()
    old = old.replace("\\n", "\n")
    assert text.count(old) == 1, old
    (d / "circ.c").write_text(text.replace(old, new))
    lib = str(d / "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
                           str(d / "oracle.c"), str(d / "denoise.c"), str(d / "circ.c"), "-o", lib, "-lm"])
    # point the oracle modules at the edited library for the duration of the pin
    mutant = ctypes.CDLL(lib)
    monkeypatch.setattr(O, "_lib", mutant)
    monkeypatch.setattr(C, "_ready", False)
    for name_, (res, args) in _base_sigs().items():
        f = getattr(mutant, name_)
        f.restype, f.argtypes = res, args
    with pytest.raises(AssertionError):
        pin()
    monkeypatch.setattr(C, "_ready", False)


def _base_sigs():
    """ctypes signatures of the Cartesian oracle entry points the pins use."""
    G = ctypes.POINTER(O.OraGrid)
    LP = ctypes.POINTER(O.OraLaser)
    dp = ctypes.POINTER(ctypes.c_double)
    return {"ora_field_step": (None, [G, dp, dp, dp]),
            "ora_field_step_laser": (None, [G, dp, dp, dp, LP, ctypes.c_double]),
            "ora_pd_coeffs": (ctypes.c_int, [dp, ctypes.c_int, dp, dp, dp]),
            "ora_boris": (None, [dp, dp, dp, ctypes.c_double, ctypes.c_double])}


def _energy_growth(nz, nr, dz, dr, dt, steps, seed=0):
    g = C.make_grid(nz, nr, dz, dr, dt)
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((2, 3, nr, nz)) + 1j * rng.standard_normal((2, 3, nr, nz))
    B = rng.standard_normal((2, 3, nr, nz)) + 1j * rng.standard_normal((2, 3, nr, nz))
    E[0], B[0] = E[0].real, B[0].real
    E, B = np.ascontiguousarray(E), np.ascontiguousarray(B)
    e0 = C.field_energy(g, E, B)
    for _ in range(steps):
        E, B = C.field_step(g, E, B)
    return C.field_energy(g, E, B) / e0


@pytest.mark.parametrize("dz,dr", [(0.05, 0.2), (0.2, 0.2), (0.2, 0.1)])
def test_time_step_bound_keeps_random_fields_bounded(dz, dr):
    """The descriptor's bound dt <= 0.95 / sqrt(1/dz^2 + 4/dr^2): random
    fields of both modes stay bounded for 3000 steps at the bound, and the
    same test does see a growth above the scheme's limit."""
    bound = 0.95 / math.sqrt(1 / dz ** 2 + 4 / dr ** 2)
    assert _energy_growth(16, 8, dz, dr, bound, 3000) < 1.5
    if dz < dr:
        over = 1.5 / math.sqrt(1 / dz ** 2 + 1 / dr ** 2)
        ratio = _energy_growth(16, 8, dz, dr, over, 400)
        assert not ratio < 100.0
