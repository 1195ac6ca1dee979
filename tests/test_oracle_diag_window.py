"""Pins of the oracle's diagnostics and of its moving-window driver.

ora_diag (charge, field energy, kinetic energy, max |J|) is checked against
values fixed without it: a uniform state whose sums are box volumes times
constants, momenta chosen so that gamma is an integer, and the charge of a
neutral uniform plasma.  run_lwfa (window shift, particle shift, plasma
injection and removal margins) is checked against what a window moving at c
must show: a cold plasma at rest seen from the window is exactly the lab
plasma of the window's current cells, and a vacuum pulse launched before
the window starts stays where it is in window coordinates.

Each pin is also run against copies of the oracle with a planted mistake (a
dropped cell volume, gamma in place of gamma - 1, the plasma injected one
cell off, ...), built on the CPU from edited sources; every planted
mistake must make the pin fail.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import oracle_mutant


# ---------------------------------------------------------------- ora_diag
def pin_diag(Om):
    """ora_diag against closed forms; raises AssertionError on a mismatch."""
    n, d = (6, 5, 4), (0.2, 0.3, 0.4)
    g = Om.make_grid(n, d, 0.05)
    volume = n[0] * d[0] * n[1] * d[1] * n[2] * d[2]          # box volume, 0.72
    E = Om.zeros_field(g)
    B = Om.zeros_field(g)
    e0, b0 = (1.0, -2.0, 3.0), (0.5, -1.0, 2.0)
    for c in range(3):
        E[c] = e0[c]
        B[c] = b0[c]
    # momenta with integer gamma: |u|^2 = gamma^2 - 1
    u = np.array([[0.0, 1.0, 2.0, 0.0],
                  [0.0, 1.0, 2.0, 0.0],
                  [0.0, 1.0, 4.0, math.sqrt(8.0)]])       # gamma = 1, 2, 5, 3
    w = np.array([0.5, 0.25, 2.0, 1.0])
    J = Om.zeros_field(g)
    J[1, 2, 3, 4] = -7.5
    J[0, 1, 1, 1] = 6.25
    J[2, 0, 0, 0] = 7.25
    dv = volume / (n[0] * n[1] * n[2])
    for q, m in ((-1.0, 1.0), (2.0, 3.0)):
        out = Om.diag(g, u, w, E, B, J, q=q, m=m)
        assert abs(out["charge"] - q * w.sum() * dv) < 1e-14
        # uniform fields: energy density 1/2 (|E|^2 + |B|^2) = 1/2 (14 + 5.25) over the whole box
        assert abs(out["e_field"] - 0.5 * 19.25 * volume) < 1e-12
        # sum w (gamma - 1) = 0.5*0 + 0.25*1 + 2*4 + 1*2 = 10.25
        assert abs(out["e_kin"] - m * 10.25 * dv) < 1e-12
        assert out["max_abs_J"] == 7.5
    assert Om.diag(g, u, w, E, B, None)["max_abs_J"] == 0.0
    # a neutralising uniform plasma of density n0 = 1.5 at 8 per cell carries -n0 V
    ppc, n0 = 8, 1.5
    npart = ppc * n[0] * n[1] * n[2]
    out = Om.diag(g, np.zeros((3, npart)), np.full(npart, n0 / ppc), Om.zeros_field(g), Om.zeros_field(g))
    assert abs(out["charge"] + n0 * volume) < 1e-12
    assert out["e_kin"] == 0.0 and out["e_field"] == 0.0


def test_ora_diag_matches_closed_forms():
    pin_diag(O)


# ---------------------------------------------------------------- run_lwfa
def _window_setup(Om, nx=24):
    g = Om.make_grid((nx, 4, 3), (0.25, 0.5, 0.5), 0.25, solver="pd", xbc=1)
    P = Om.make_plasma(x_start=5, ramp=7, n_plateau=1.25, ppc=(2, 1, 2))
    # no laser: the source is gated off (t_end < 0)
    L = Om.make_laser(a0=1.0, omega0=1.508, waist=1.0, fwhm=1.0, t_peak=1.0, t_end=-1.0, yc=1.0, zc=0.75, src_x=2)
    return g, P, L


def pin_window_cold_plasma(Om):
    """Cold plasma at rest, window moving from step 0: after k steps the
    particles are exactly the lab plasma over window cells [3, nx - 4]."""
    nx = 24
    g, P, L = _window_setup(Om, nx)
    for k in (1, 7, 30):     # 30 > nx: every particle loaded at start has left
        out = Om.run_lwfa(g, P, L, nsteps=k, window_start=0)
        assert out["shift"] == k
        xw, ww, idw = Om.inject(g, P, k, 3, nx - 3)
        order = np.argsort(out["id"])
        worder = np.argsort(idw)
        assert np.array_equal(out["id"][order], idw[worder])
        assert np.array_equal(out["x"][:, order], xw[:, worder])
        assert np.array_equal(out["w"][order], ww[worder])
        assert not np.any(out["u"]) and not np.any(out["E"]) and not np.any(out["B"])
        # the plasma edge: lab cell x_start = 5 is window cell 5 - k
        lab_first = 5 - k
        assert out["x"][0].min() >= max(3, lab_first) * g.d[0]
    # window not moving: nothing is added, the set is the initial one minus the back margin
    out = Om.run_lwfa(g, P, L, nsteps=4, window_start=100)
    x0, w0, id0 = Om.inject(g, P, 0, 3, nx - 3)
    assert out["shift"] == 0 and np.array_equal(np.sort(out["id"]), np.sort(id0))


def pin_window_vacuum_pulse(Om):
    """A plane pulse launched before the window starts keeps its window
    position once the window moves at c (perfect dispersion at c dt = dx
    propagates axial waves exactly), and it is the exact discrete wave
    E_y(i) = e((W - i + src) dt) of the step W at which the window starts."""
    nx = 96
    g = Om.make_grid((nx, 4, 4), (0.25, 0.5, 0.5), 0.25, solver="pd", xbc=1)
    P = Om.make_plasma(x_start=1e9, ramp=0.0, n_plateau=0.0, ppc=(1, 1, 1))
    src = 4
    L = Om.make_laser(a0=1.5, omega0=1.508, waist=1e12, fwhm=1.0, t_peak=4.0, t_end=9.0, yc=1.0, zc=1.0, src_x=src)
    W = 40                   # the state after W steps (t = 10 > t_end) ...
    ref = Om.run_lwfa(g, P, L, nsteps=W, window_start=10 ** 9)
    # ... and 25 steps more, each followed by a window move
    out = Om.run_lwfa(g, P, L, nsteps=W + 25, window_start=W + 1)
    assert out["shift"] == 25 and out["x"].shape[1] == 0
    want = np.array([Om.laser_e(L, (W - i + src) * g.dt) for i in range(nx)])
    amp = np.abs(want).max()
    ey = out["E"][1, 0, 0, :]
    # behind the source plane the moved window holds what had entered past it
    assert np.abs(ey[src:] - want[src:]).max() < 1e-8 * amp
    assert np.abs(out["E"] - ref["E"]).max() < 1e-8 * amp
    assert np.abs(out["B"] - ref["B"]).max() < 1e-8 * amp


def test_run_lwfa_window_reproduces_the_lab_plasma():
    pin_window_cold_plasma(O)


def test_run_lwfa_window_keeps_a_vacuum_pulse_in_place():
    pin_window_vacuum_pulse(O)


# ---------------------------------------------------------------- planted mistakes
def _mutant(tmp_path, name, c_edit=None, py_edit=None):
    return oracle_mutant(tmp_path, name, c_edit, py_edit)


MUTANTS = [
    ("diag_no_dv_charge", pin_diag, ("charge += q * w[p] * dv;", "charge += q * w[p];"), None),
    ("diag_gamma_not_minus_one", pin_diag,
     ("ek += m * w[p] * (sqrt(1.0 + u2) - 1.0) * dv;", "ek += m * w[p] * sqrt(1.0 + u2) * dv;"), None),
    ("diag_no_half", pin_diag,
     ("ef += 0.5 * (E[f] * E[f] + B[f] * B[f]) * dv;", "ef += (E[f] * E[f] + B[f] * B[f]) * dv;"), None),
    ("diag_signed_max", pin_diag,
     ("if (J && fabs(J[f]) > mj) mj = fabs(J[f]);", "if (J && J[f] > mj) mj = J[f];"), None),
    ("diag_e_only", pin_diag,
     ("ef += 0.5 * (E[f] * E[f] + B[f] * B[f]) * dv;", "ef += 0.5 * (E[f] * E[f]) * dv;"), None),
    ("window_inject_one_cell_ahead", pin_window_cold_plasma, None,
     ("inject(g, P, shift, nx - 1 - inject_hi, nx - inject_hi)", "inject(g, P, shift, nx - inject_hi, nx + 1 - inject_hi)")),
    ("window_kill_margin_short", pin_window_cold_plasma, None,
     ("k = (x[0] >= kill_lo * g.d[0])", "k = (x[0] >= (kill_lo - 1) * g.d[0])")),
    ("window_particles_not_shifted", pin_window_cold_plasma, None, ("            x[0] -= g.d[0]\n", "")),
    ("window_inject_lab_cell_off", pin_window_cold_plasma, None,
     ("inject(g, P, shift, nx - 1 - inject_hi, nx - inject_hi)",
      "inject(g, P, shift + 1, nx - 1 - inject_hi, nx - inject_hi)")),
    ("window_fields_shift_backwards", pin_window_vacuum_pulse,
     ("for (int64_t i = 0; i + 1 < nx; ++i) row[i] = row[i + 1];\n                row[nx - 1] = 0.0;",
      "for (int64_t i = nx - 1; i > 0; --i) row[i] = row[i - 1];\n                row[0] = 0.0;"), None),
    ("window_fields_not_shifted", pin_window_vacuum_pulse, None,
     ("            E, B = window_shift(g, E, B)\n", "")),
    ("window_laser_one_step_early", pin_window_vacuum_pulse, None, ("        t = n * g.dt\n", "        t = (n + 1) * g.dt\n")),
    ("window_laser_off", pin_window_vacuum_pulse, None,
     ("L if (shift == 0 and t <= L.t_end) else None", "None")),
]


@pytest.mark.parametrize("name,pin,c_edit,py_edit", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_rejects_planted_mistake(tmp_path, name, pin, c_edit, py_edit):
    mod = _mutant(tmp_path, name, c_edit, py_edit)
    with pytest.raises(AssertionError):
        pin(mod)
