"""Pins of the oracle's transverse perfectly matched layer (Section 3.1 runs
its Cartesian box inside a 16-layer PML; the formulation, a convolutional
PML with a graded conductivity, is stated in oracle/oracle.c).

Each pin fixes the layer by something other than the oracle itself:

- the conductivity profile against its closed form and its symmetry;
- with zero conductivity the layer step is the plain field step with zero
  fields beyond the transverse edges, bit for bit;
- in a layer of constant conductivity sigma a plane wave decays as
  exp(-sigma t) while it crosses it, whatever its frequency -- the defining
  property of a matched layer (stretched coordinate 1 + sigma / (i omega));
  checked for both polarisations along y and along z, which exercises all
  eight auxiliary arrays;
- a graded 16-layer wall reflects a normally incident pulse below 2e-5 of
  its amplitude, and an obliquely incident cylindrical pulse of the
  perfect-dispersion solver below 2e-5 of the peak, judged against the same
  pulse on a periodic box large enough that nothing comes back in time;
  without conductivity the same walls reflect it almost fully;
- moving the window commutes with the field steps: shifting the fields and
  the auxiliary arrays after some steps gives, bit for bit, what shifting
  the initial fields first gives;
- in the laser-wakefield driver, particles whose transverse cell lies in
  the layer are never pushed.

Each pin is also run against copies of the oracle with a planted mistake;
every one must make its pin fail.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import oracle_mutant


# ---------------------------------------------------------------- profile
def pin_profile(Om):
    n, d, L = (4, 40, 48), (0.25, 0.5, 0.4), 8
    g = Om.make_grid(n, d, 0.1, yzbc=3)
    P = Om.make_pml(g, layers=L)
    for a in (1, 2):
        smax = 0.8 * 4.0 / d[a]
        na = n[a]
        for p in range(L - 1, na - L + 1):
            assert Om.pml_sigma(P, a, na, float(p)) == 0.0, (a, p)
        assert abs(Om.pml_sigma(P, a, na, -1.0) - smax) <= 1e-12 * smax
        assert abs(Om.pml_sigma(P, a, na, float(na)) - smax) <= 1e-12 * smax
        # half way through the layer: (1/2)^3 of the maximum
        assert abs(Om.pml_sigma(P, a, na, L - 1 - L / 2) - smax / 8) <= 1e-12 * smax
        assert abs(Om.pml_sigma(P, a, na, na - L + L / 4) - smax / 64) <= 1e-12 * smax
        for p2 in range(-2, 2 * na + 1):
            p = 0.5 * p2
            s, s_mirror = Om.pml_sigma(P, a, na, p), Om.pml_sigma(P, a, na, na - 1 - p)
            assert abs(s - s_mirror) <= 1e-12 * smax, (a, p)


def test_profile():
    pin_profile(O)


# ---------------------------------------------------------------- zero conductivity
def _random_fields(g, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(O._fshape(g)), rng.standard_normal(O._fshape(g))


def pin_zero_sigma(Om):
    for solver in ("yee", "pd"):
        g = Om.make_grid((8, 10, 12), (0.25, 0.5, 0.5), 0.2, solver=solver, yzbc=3)
        P = Om.make_pml(g, layers=4, sigma_max=0.0)
        E, B = _random_fields(g, 7)
        J = np.random.default_rng(8).standard_normal(E.shape)
        Ea, Ba, psi = E, B, Om.zeros_psi(g)
        Eb, Bb = E, B
        for _ in range(3):
            Ea, Ba, psi = Om.pml_field_step(g, P, Ea, Ba, psi, J)
            Eb, Bb = Om.field_step(g, Eb, Bb, J)
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb), solver
        # the laser form of the step, too
        L = Om.make_laser(1.0, 6.0, 1.5, 1.0, 0.5, 2.0, 2.5, 3.0, 2)
        Ea, Ba, psi = E, B, Om.zeros_psi(g)
        Eb, Bb = E, B
        for s in range(3):
            Ea, Ba, psi = Om.field_step_laser_pml(g, Ea, Ba, J, L, s * g.dt, P, psi)
            Eb, Bb = Om.field_step_laser(g, Eb, Bb, J, L, s * g.dt)
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb), solver


def test_zero_sigma_is_the_plain_step():
    pin_zero_sigma(O)


# ---------------------------------------------------------------- constant conductivity
# A plane pulse travelling +axis: axis y, (E_z, B_x) or (E_x, -B_z); axis z,
# (E_x, B_y) or (E_y, -B_x).
_POL = {(1, "a"): ((2, 1.0), (0, 1.0)), (1, "b"): ((0, 1.0), (2, -1.0)),
        (2, "a"): ((0, 1.0), (1, 1.0)), (2, "b"): ((1, 1.0), (0, -1.0))}


def _plane_pulse(Om, g, axis, pol, c0, w):
    n, d = int(g.n[axis]), g.d[axis]
    (ce, se), (cb, sb) = _POL[(axis, pol)]
    E, B = Om.zeros_field(g), Om.zeros_field(g)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    pos = np.arange(n) * d
    E[ce][...] = se * np.exp(-0.5 * ((pos - c0) / w) ** 2).reshape(shape)
    B[cb][...] = sb * np.exp(-0.5 * ((pos + 0.5 * d - c0) / w) ** 2).reshape(shape)
    return E, B


def _axis_slice(axis, lo, hi):
    sl = [slice(None)] * 4
    sl[3 - axis] = slice(lo, hi)
    return tuple(sl)


def pin_uniform_rate(Om, sigma=0.2):
    n, d, L = 400, 0.5, 100
    for axis in (1, 2):
        for pol in "ab":
            nn = [2, 2, 2]
            nn[axis] = n
            g = Om.make_grid(nn, (0.5, 0.5, 0.5), 0.2, yzbc=axis)
            P = Om.make_pml(g, layers=L, sigma_max=sigma, grade=0.0, axes=(axis,))
            c0 = 0.5 * n * d                       # pulse starts at the centre
            E, B = _plane_pulse(Om, g, axis, pol, c0, 4 * d)
            psi = Om.zeros_psi(g)
            t_in = (n - L) * d - c0                # its peak reaches the layer
            t1, t2 = t_in + 5.0, t_in + 25.0
            i1, i2 = int(round(t1 / g.dt)), int(round(t2 / g.dt))
            peak = {}
            for s in range(1, i2 + 1):
                E, B, psi = Om.pml_field_step(g, P, E, B, psi)
                if s in (i1, i2):
                    peak[s] = np.abs(E[_axis_slice(axis, n - L, n)]).max()
            rate = np.log(peak[i1] / peak[i2]) / (t2 - t1)
            assert abs(rate - sigma) <= 0.015 * sigma, (axis, pol, rate)


def test_uniform_layer_attenuates_at_sigma():
    pin_uniform_rate(O)


# ---------------------------------------------------------------- graded wall, normal incidence
def pin_normal_reflection(Om):
    n, d, L = 200, 0.5, 16
    for axis, pol in ((1, "a"), (2, "b")):
        nn = [2, 2, 2]
        nn[axis] = n
        g = Om.make_grid(nn, (0.5, 0.5, 0.5), 0.2, yzbc=axis)
        P = Om.make_pml(g, layers=L, axes=(axis,))
        Pz = Om.make_pml(g, layers=L, sigma_max=0.0, axes=(axis,))
        nl = list(nn)
        nl[axis] = 4 * n                              # periodic, nothing returns in time
        gl = Om.make_grid(nl, (0.5, 0.5, 0.5), 0.2)
        c0 = 0.5 * n * d
        E, B = _plane_pulse(Om, g, axis, pol, c0, 4 * d)
        Ez, Bz, psi, psz = E, B, Om.zeros_psi(g), Om.zeros_psi(g)
        El, Bl = _plane_pulse(Om, gl, axis, pol, c0 + 1.5 * n * d, 4 * d)
        inner, inner_l = _axis_slice(axis, L, n - L), _axis_slice(axis, 3 * n // 2 + L, 5 * n // 2 - L)
        err = err_pec = 0.0
        for _ in range(int((0.5 * n * d + 2 * L * d + 10.0) / g.dt)):
            E, B, psi = Om.pml_field_step(g, P, E, B, psi)
            Ez, Bz, psz = Om.pml_field_step(g, Pz, Ez, Bz, psz)
            El, Bl = Om.field_step(gl, El, Bl)
            err = max(err, np.abs(E[inner] - El[inner_l]).max())
            err_pec = max(err_pec, np.abs(Ez[inner] - El[inner_l]).max())
        assert err < 2e-5, (axis, pol, err)
        assert err_pec > 0.5, (axis, pol, err_pec)


def test_graded_wall_normal_reflection():
    pin_normal_reflection(O)


# ---------------------------------------------------------------- graded wall, oblique incidence (PD)
def _cyl_pulse(Om, g, c, w):
    y = (np.arange(int(g.n[1])) + 0.5) * g.d[1]
    z = (np.arange(int(g.n[2])) + 0.5) * g.d[2]
    B = Om.zeros_field(g)
    B[0][...] = np.exp(-((y[None, :, None] - c) ** 2 + (z[:, None, None] - c) ** 2) / w ** 2)
    return Om.zeros_field(g), B


def pin_oblique_reflection(Om):
    nt, L, nref, d, dt = 48, 16, 72, (0.25, 0.5, 0.5), 0.25
    g = Om.make_grid((4, nt, nt), d, dt, solver="pd", yzbc=3)
    P = Om.make_pml(g, layers=L)
    Pz = Om.make_pml(g, layers=L, sigma_max=0.0)
    gr = Om.make_grid((4, nref, nref), d, dt, solver="pd")
    E, B = _cyl_pulse(Om, g, 0.25 * nt, 1.5)
    Ez, Bz, psi, psz = E, B, Om.zeros_psi(g), Om.zeros_psi(g)
    Er, Br = _cyl_pulse(Om, gr, 0.25 * nref, 1.5)
    o = (nref - nt) // 2
    inner = (slice(None), slice(L, nt - L), slice(L, nt - L))
    inner_r = (slice(None), slice(o + L, o + nt - L), slice(o + L, o + nt - L))
    err = err_pec = peak = 0.0
    for _ in range(int(24.0 / dt)):
        E, B, psi = Om.pml_field_step(g, P, E, B, psi)
        Ez, Bz, psz = Om.pml_field_step(g, Pz, Ez, Bz, psz)
        Er, Br = Om.field_step(gr, Er, Br)
        err = max(err, np.abs(E[inner] - Er[inner_r]).max())
        err_pec = max(err_pec, np.abs(Ez[inner] - Er[inner_r]).max())
        peak = max(peak, np.abs(Er[inner_r]).max())
    assert err < 2e-5 * peak, (err, peak)
    assert err_pec > 0.1 * peak, (err_pec, peak)


def test_graded_wall_oblique_reflection_pd():
    pin_oblique_reflection(O)


# ---------------------------------------------------------------- window shift
def pin_window_commutes(Om):
    n, L = (48, 40, 24), 8
    g = Om.make_grid(n, (0.25, 0.5, 0.5), 0.25, solver="pd", xbc=1, yzbc=3)
    P = Om.make_pml(g, layers=L)
    E, B = Om.zeros_field(g), Om.zeros_field(g)
    x = np.arange(n[0])[None, None, :]
    y = np.arange(n[1])[None, :, None]
    z = np.arange(n[2])[:, None, None]
    r2 = ((x - 24) / 2.0) ** 2 + ((y - (L + 2)) / 2.0) ** 2 + ((z - 12) / 3.0) ** 2
    blob = np.where(np.abs(x - 24) <= 3, np.exp(-r2), 0.0)       # exactly zero near the x ends
    E[1] = blob
    B[2] = 0.5 * blob
    n1, n2 = 4, 2
    Ea, Ba, pa = E, B, Om.zeros_psi(g)
    for _ in range(n1):
        Ea, Ba, pa = Om.pml_field_step(g, P, Ea, Ba, pa)
    assert np.abs(pa).max() > 1e-3                                # the layer has taken some of it
    Ea, Ba = Om.window_shift(g, Ea, Ba)
    pa = Om.pml_window_shift(g, pa)
    for _ in range(n2):
        Ea, Ba, pa = Om.pml_field_step(g, P, Ea, Ba, pa)
    Eb, Bb = Om.window_shift(g, E, B)
    pb = Om.zeros_psi(g)
    for _ in range(n1 + n2):
        Eb, Bb, pb = Om.pml_field_step(g, P, Eb, Bb, pb)
    assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb) and np.array_equal(pa, pb)


def test_window_shift_commutes_with_the_layer():
    pin_window_commutes(O)


# ---------------------------------------------------------------- particles in the layer
def pin_lwfa_layer_kill(Om):
    n, L = (16, 12, 10), 3
    g = Om.make_grid(n, (0.25, 0.5, 0.5), 0.25, solver="pd", xbc=1, yzbc=3)
    P = Om.make_plasma(4.0, 0.0, 1.0, (1, 1, 1))
    laser = Om.make_laser(0.0, 6.0, 1.0, 1.0, 0.5, -1.0, 3.0, 2.5, 2)     # never on
    pml = Om.make_pml(g, layers=L)
    out = Om.run_lwfa(g, P, laser, 3, 1000, pml=pml)
    # a cold plasma in vacuum fields stays where it was loaded: one particle
    # per cell x >= 4 .. nx - 4 in the transverse cells L .. n - L - 1
    ids = sorted(((X * n[1] + j) * n[2] + k) for X in range(4, n[0] - 3)
                 for j in range(L, n[1] - L) for k in range(L, n[2] - L))
    assert sorted(out["id"].tolist()) == ids
    assert np.abs(out["u"]).max() == 0.0


def test_lwfa_removes_particles_in_the_layer():
    pin_lwfa_layer_kill(O)


# ---------------------------------------------------------------- planted mistakes
MUTANTS = [
    ("profile_asymmetric", pin_profile,
     ("double lo = (L - 1.0 - p) / L, hi", "double lo = (L - p) / L, hi"), None),
    ("profile_quadratic", pin_profile, None, ("sigma_max=None, grade: float = 3.0", "sigma_max=None, grade: float = 2.0")),
    ("b_update_drops_x_curl_term", pin_zero_sigma,
     ("tmp[nc + f] = dzEx - dsmooth(g, Ez, 0, i, j, k);", "tmp[nc + f] = dzEx;"), None),
    ("e_update_sign", pin_zero_sigma,
     ("tmp[f] = dyBz - dzBy;\n                tmp[nc + f] = dzBx - dback(g, Bz, 0, i, j, k);\n"
      "                tmp[2 * nc + f] = dback(g, By, 0, i, j, k) - dyBx;\n            }\n"
      "    for (int64_t f = 0; f < 3 * nc; ++f) E[f] += g->dt * (tmp[f] - (J ? J[f] : 0.0));\n    free(tmp);\n}\n\n"
      "/* One field step with the transverse layer",
      "tmp[f] = dzBy - dyBz;\n                tmp[nc + f] = dzBx - dback(g, Bz, 0, i, j, k);\n"
      "                tmp[2 * nc + f] = dback(g, By, 0, i, j, k) - dyBx;\n            }\n"
      "    for (int64_t f = 0; f < 3 * nc; ++f) E[f] += g->dt * (tmp[f] - (J ? J[f] : 0.0));\n    free(tmp);\n}\n\n"
      "/* One field step with the transverse layer"), None),
    ("b_psi_half_rate", pin_uniform_rate,
     ("double b = exp(-sigma * dt);\n    double p = b", "double b = exp(-0.5 * sigma * dt);\n    double p = b"), None),
    ("e_psi_sign", pin_uniform_rate,
     ("*psi = b * (*psi) + (b - 1.0) * D;", "*psi = b * (*psi) + (1.0 - b) * D;"), None),
    ("psi_arrays_shared", pin_uniform_rate,
     ("double dzEx = stretch_b(psi + 2 * nc + f,", "double dzEx = stretch_b(psi + nc + f,"), None),
    ("e_psi_missing_on_one_term", pin_uniform_rate,
     ("double dyBx = stretch(psi + 3 * nc + f, dback(g, Bx, 1, i, j, k), sy, g->dt);",
      "double dyBx = dback(g, Bx, 1, i, j, k);"), None),
    ("b_psi_split_per_half_step", pin_normal_reflection,
     ("if (store) *psi = p;", "*psi = p;"), None),
    ("e_psi_at_half_positions", pin_normal_reflection,
     ("double sy = pml_sigma(P, 1, g->n[1], (double)j), sz = pml_sigma(P, 2, g->n[2], (double)k);",
      "double sy = pml_sigma(P, 1, g->n[1], (double)j + 0.5), sz = pml_sigma(P, 2, g->n[2], (double)k + 0.5);"),
     None),
    ("psi_not_moved_with_window", pin_window_commutes,
     ("for (int a = 0; a < 8; ++a) shift_down_x(g, psi + a * nc);", "(void)nc;"), None),
    ("layer_kill_one_cell_short", pin_lwfa_layer_kill, None,
     ("k &= (c >= lay) & (c < int(g.n[a]) - lay)", "k &= (c >= lay - 1) & (c < int(g.n[a]) - lay)")),
]


@pytest.mark.parametrize("name,pin,c_edit,py_edit", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_rejects_planted_mistake(tmp_path, name, pin, c_edit, py_edit):
    mod = oracle_mutant(tmp_path, name, c_edit, py_edit)
    with pytest.raises(AssertionError):
        pin(mod)
