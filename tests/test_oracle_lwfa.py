"""Pins of the oracle's laser-wakefield boundaries: laser source, moving
window and plasma loading along a density ramp."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _laser(**kw):
    base = dict(a0=2.0, omega0=1.508, waist=1e9, fwhm=1.0, t_peak=4.0, t_end=8.0, yc=0.0, zc=0.0, src_x=4)
    base.update(kw)
    return O.make_laser(**base)


def test_laser_field_has_no_dc_and_the_right_amplitude():
    L = _laser()
    ts = np.linspace(-20, 30, 200001)
    e = np.array([O.laser_e(L, t) for t in ts])
    # E = -dA/dt with A(+-inf) = 0: no net area
    assert abs(np.trapezoid(e, ts)) < 1e-9 * np.abs(e).max()
    # many-cycle pulse: peak E ~ a0 omega0
    Ll = _laser(fwhm=60.0, t_peak=100.0, omega0=2.0)
    ts = np.linspace(80, 120, 40001)
    e = np.array([O.laser_e(Ll, t) for t in ts])
    assert abs(np.abs(e).max() / (2.0 * 2.0) - 1) < 2e-3
    # intensity envelope FWHM: cycle-averaged e^2 falls to half at t_peak +- fwhm/2
    half = np.mean([O.laser_e(Ll, 130 + s) ** 2 for s in np.linspace(-math.pi / 2, math.pi / 2, 201)])
    peak = np.mean([O.laser_e(Ll, 100 + s) ** 2 for s in np.linspace(-math.pi / 2, math.pi / 2, 201)])
    assert abs(half / peak - 0.5) < 0.02


def _plane_wave_grid(nx=128):
    return O.make_grid((nx, 4, 4), (0.25, 0.5, 0.5), 0.25, solver="pd", xbc=1)


def test_tfsf_source_launches_the_exact_discrete_plane_wave_forward_only():
    """PD at c dt = dx propagates axial waves exactly, so a plane-wave source must
    give E_y(i, n) = e((n - i + src) dt) ahead of the plane and nothing behind it."""
    g = _plane_wave_grid()
    L = _laser(waist=1e12, yc=1.0, zc=1.0)
    E = O.zeros_field(g)
    B = O.zeros_field(g)
    N = 90
    for n in range(N):
        E, B = O.field_step_laser(g, E, B, None, L, n * g.dt)
    ey = E[1, 0, 0, :]
    i = np.arange(128)
    want = np.array([O.laser_e(L, (N - k + 4) * g.dt) for k in i])
    amp = np.abs(want).max()
    # the source switches on at t = 0, where the envelope is exp(-22): the wave
    # front differs from the ever-running pulse by that much
    assert np.abs(ey[4:] - want[4:]).max() < 1e-8 * amp
    assert np.abs(E[:, :, :, :3]).max() < 1e-11 * amp
    assert np.abs(B[:, :, :, :3]).max() < 1e-11 * amp
    assert np.abs(E[0]).max() == 0 and np.abs(E[2]).max() == 0


def test_moving_window_keeps_a_vacuum_pulse_stationary():
    g = _plane_wave_grid()
    L = _laser(waist=1e12, yc=1.0, zc=1.0)
    E = O.zeros_field(g)
    B = O.zeros_field(g)
    for n in range(40):
        E, B = O.field_step_laser(g, E, B, None, L, n * g.dt)
    E0, B0 = E.copy(), B.copy()
    for _ in range(30):   # source off; the window moves with the pulse
        E, B = O.field_step_laser(g, E, B, None, None, 0.0)
        E, B = O.window_shift(g, E, B)
    assert np.allclose(E, E0, atol=1e-11 * np.abs(E0).max())
    assert np.allclose(B, B0, atol=1e-11 * np.abs(B0).max())


def test_plasma_loading_matches_the_profile_integral_and_the_lab_frame():
    g = O.make_grid((40, 6, 5), (0.25, 0.5, 0.5), 0.25, solver="pd", xbc=1)
    P = O.make_plasma(x_start=8, ramp=10, n_plateau=1.5, ppc=(2, 2, 2))
    x, w, ids = O.inject(g, P, 0, 0, 40)
    # midpoint rule on the sub-lattice is exact for a profile linear between lattice-cell faces
    integral = 1.5 * ((40 - 8 - 10) + 10 / 2)
    assert abs(w.sum() - integral * 6 * 5) < 1e-9
    assert x[0].min() >= 8 * 0.25 and len(np.unique(ids)) == len(ids)
    # the same lab cells loaded after the window moved 5 cells
    xs, ws, idss = O.inject(g, P, 5, 0, 35)
    a = {int(k): (xx, ww) for k, xx, ww in zip(ids, x[0], w)}
    for k, xx, ww in zip(idss, xs[0], ws):
        xa, wa = a[int(k)]
        assert abs((xx + 5 * 0.25) - xa) < 1e-12 and abs(ww - wa) < 1e-15
    assert O.density(P, 7.9) == 0.0 and abs(O.density(P, 13.0) - 0.75) < 1e-15 and O.density(P, 30) == 1.5


def test_lwfa_run_conserves_charge_apart_from_window_traffic():
    g = O.make_grid((32, 8, 8), (0.25, 0.5, 0.5), 0.25, solver="pd", xbc=1)
    P = O.make_plasma(x_start=6, ramp=6, n_plateau=1.0, ppc=(1, 1, 1))
    L = _laser(waist=1.5, yc=2.0, zc=2.0, t_end=4.0, t_peak=2.0)
    out = O.run_lwfa(g, P, L, nsteps=10, window_start=100)
    x, w = out["x"], out["w"]
    # window never moved: particles only leave through the kill margins
    x0, w0, _ = O.inject(g, P, 0, 0, 32 - 3)
    assert len(w) <= len(w0) and np.all(np.isfinite(out["E"]))
    assert np.abs(out["E"][1]).max() > 0.1     # the laser entered
