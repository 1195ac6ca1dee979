"""Pins of the laser group velocity the oracle's two solvers give a plane
pulse along x (the paper's Section 1 and 3.3 mechanism: the Yee scheme's
axial dispersion slows the pulse; the perfect-dispersion curl at c dt = dx
does not).  The centroid of the pulse's energy must move at exactly c under
perfect dispersion, and, under Yee, at the spectral average of the Yee
group velocity d omega/dk = cos(k dx/2)/cos(omega dt/2) (from the discrete
dispersion relation sin(omega dt/2)/dt = sin(k dx/2)/dx) over the pulse's
power spectrum, to 5% of the slowdown."""
import math

import numpy as np

from oracle import diagnostics as DG
from oracle import oracle as O

D = (0.25, 0.5, 0.5)
NX = 320
OMEGA0 = 2 * math.pi / (0.25 / 0.06)


def plane_pulse_run(solver, dt, t_from=30.0, t_to=70.0, every=5):
    """Oracle run of the plane C1 pulse; returns (times, centroids, E at t_from)."""
    g = O.make_grid((NX, 4, 4), D, dt, solver=solver, xbc=1)
    L = O.make_laser(a0=1.0, omega0=OMEGA0, waist=1e12, fwhm=2.5, t_peak=10.0, t_end=20.0, yc=1.0, zc=1.0, src_x=2)
    E, B = O.zeros_field(g), O.zeros_field(g)
    ts, xc, snap = [], [], None
    total = int(round(t_to / dt))
    for n in range(total):
        t = n * dt
        E, B = O.field_step_laser(g, E, B, None, L if t <= L.t_end else None, t)
        tt = (n + 1) * dt
        if tt >= t_from and (n + 1) % every == 0:
            m = DG.field_moments(E, B, D, transverse_only=True)
            ts.append(tt)
            xc.append(m[1] / m[0])
            if snap is None:
                snap = E[1, 0, 0, :].copy()
    return np.array(ts), np.array(xc), snap


def yee_dt():
    return 0.98 / math.sqrt(sum(1.0 / (v * v) for v in D))


def test_perfect_dispersion_pulse_moves_at_c():
    ts, xc, _ = plane_pulse_run("pd", D[0])
    v = np.polyfit(ts, xc, 1)[0]
    assert abs(v - 1.0) < 1e-10, v


def test_yee_pulse_moves_at_the_spectral_group_velocity():
    dt = yee_dt()
    ts, xc, ey = plane_pulse_run("yee", dt)
    v = np.polyfit(ts, xc, 1)[0]
    M = 1 << 14
    F = np.fft.rfft(ey, n=M)
    k = 2 * np.pi * np.fft.rfftfreq(M, d=D[0])
    w = 2.0 / dt * np.arcsin(dt / D[0] * np.sin(k * D[0] / 2))
    vg = np.cos(k * D[0] / 2) / np.cos(w * dt / 2)
    P = np.abs(F) ** 2
    pred = (P * vg).sum() / P.sum()
    assert 1.0 - pred > 5e-3                      # a slowdown of order 1%
    assert abs(v - pred) < 0.05 * (1.0 - pred), (v, pred)
    # and not the carrier's group velocity alone (the pulse is a few cycles long)
    w0 = 2.0 / dt * math.asin(dt / D[0] * math.sin(OMEGA0 * D[0] / 2))
    assert abs(v - math.cos(OMEGA0 * D[0] / 2) / math.cos(w0 * dt / 2)) > 0.5 * abs(v - pred)
