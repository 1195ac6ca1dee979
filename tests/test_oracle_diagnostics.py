"""Pins of the oracle's run diagnostics (oracle/diagnostics.py) against
closed forms: bilinear interpolation reproduces a linear field exactly, the
accelerating phase of a sine wake is half a wavelength, integer-gamma
momenta land in known spectrum bins, a beam built from a symmetric point set
has the product of its spreads as emittance (zero when momentum and
position are correlated), and a Gaussian pulse's energy has its centre and
width.  Each pin also rejects copies of the module with a planted mistake."""
import importlib.util
import math
import os

import numpy as np
import pytest

from oracle import diagnostics as D

HERE = os.path.dirname(D.__file__)


def pin_axis_line(M):
    n, d = (7, 9, 8), (0.25, 0.5, 0.4)
    nx, ny, nz = n
    for comp in range(6):
        sy, sz = M.YZ_STAGGER[comp]
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        y = (j + sy) * d[1]
        z = (k + sz) * d[2]
        F = 1.5 + 0.75 * y - 2.0 * z + 0.125 * i
        for yc, zc in ((1.3, 1.1), (2.0, 1.6), (3.1, 2.3)):
            got = M.axis_line(F, comp, d, yc, zc)
            want = 1.5 + 0.75 * yc - 2.0 * zc + 0.125 * np.arange(nx)
            assert np.abs(got - want).max() < 1e-12, (comp, yc, zc)


def pin_accelerating_length(M):
    dx, lam = 0.05, 6.0
    k = 2 * math.pi / lam
    xa = 12.0
    xs = (np.arange(600) + 0.5) * dx
    line = np.where(xs > xa - 1.5 * lam, np.sin(k * (xs - xa)), 0.3)
    # from inside the positive half behind xa + lam/2: the negative half-wave (xa - lam/2, xa)
    L = M.accelerating_length(line, dx, xa + 0.3 * lam)
    assert abs(L - lam / 2) < 1e-4 * lam, L
    # starting inside the negative run, the front end is x_from
    L2 = M.accelerating_length(line, dx, xa - 0.2 * lam)
    assert abs(L2 - (0.3 * lam)) < 1e-4 * lam, L2
    assert M.accelerating_length(np.abs(line) + 0.1, dx, 20.0) == 0.0


def pin_spectrum(M):
    # gamma = 1, 2, 5, 3, 2: kinetic energies 0, 1, 4, 2, 1
    u = np.array([[0.0, 1.0, 2.0, 0.0, -1.0],
                  [0.0, 1.0, 2.0, 0.0, 1.0],
                  [0.0, 1.0, 4.0, math.sqrt(8.0), -1.0]])
    w = np.array([0.5, 0.25, 2.0, 1.0, 4.0])
    charge, count = M.spectrum(u, w, -1.0, 0.125, 0, 0.0, 5.0, 5)
    assert list(count) == [1, 2, 1, 0, 1]
    assert np.allclose(charge, 0.125 * np.array([0.5, 4.25, 1.0, 0.0, 2.0]), rtol=0, atol=1e-15)
    # u_x spectrum over [-1, 2) in 3 bins: -1 -> bin 0, 0, 0 -> bin 1, 1 -> bin 2, 2 outside
    charge, count = M.spectrum(u, w, -2.0, 1.0, 1, -1.0, 2.0, 3)
    assert list(count) == [1, 2, 1]
    assert np.allclose(charge, 2.0 * np.array([4.0, 1.5, 0.25]), rtol=0, atol=1e-15)


def pin_beam_moments(M):
    a = np.array([1.0, 1.0, -1.0, -1.0])
    b = np.array([1.0, -1.0, 1.0, -1.0])
    y0, z0, sy, sz, py, pz = 40.0, 30.0, 0.5, 0.2, 0.1, 0.3
    x = np.stack([np.full(4, 5.0), y0 + sy * a, z0 + sz * b])
    u = np.stack([np.full(4, 50.0), 2.0 + py * b, -1.0 + pz * a])
    w = np.full(4, 0.25)
    m = M.beam_moments(x, u, w, -1.0, 2.0, 10.0)
    assert m["count"] == 4 and abs(m["charge"] - 2.0) < 1e-15 and abs(m["mean_ux"] - 50.0) < 1e-12
    # y with u_y independent, z with u_z independent: eps = spread(r) spread(p)
    assert abs(m["eps_ny"] - sy * py) < 1e-12 and abs(m["eps_nz"] - sz * pz) < 1e-12
    # momentum proportional to position: zero emittance (the square root of
    # a difference that cancels to round-off of var_p var_r ~ (0.35 * 0.25)^2)
    uc = np.stack([np.full(4, 50.0), 0.7 * (x[1] - y0), -0.4 * (x[2] - z0)])
    mc = M.beam_moments(x, uc, w, -1.0, 2.0, 10.0)
    assert mc["eps_ny"] < 1e-6 * 0.7 * sy * sy and mc["eps_nz"] < 1e-6 * 0.4 * sz * sz
    # selection: slow particles do not count
    u2 = u.copy()
    u2[0, :2] = 1.0
    assert M.beam_moments(x, u2, w, -1.0, 2.0, 10.0)["count"] == 2


def pin_field_moments(M):
    n, d = (400, 3, 2), (0.05, 0.5, 0.5)
    E = np.zeros((3, n[2], n[1], n[0]))
    B = np.zeros_like(E)
    x0, s = 8.0, 1.5
    xs = np.arange(n[0]) * d[0]                 # E_y sits at integer x nodes
    E[1] = np.exp(-((xs - x0) / s) ** 2)[None, None, :]
    m0, m1, m2 = M.field_moments(E, B, d)
    # energy density 1/2 exp(-2 (x - x0)^2 / s^2): integral sqrt(pi/2) s / 2 per unit area
    area = n[1] * d[1] * n[2] * d[2]
    assert abs(m0 - area * math.sqrt(math.pi / 2) * s / 2) < 1e-9 * m0
    assert abs(m1 / m0 - x0) < 1e-9
    assert abs(m2 / m0 - (m1 / m0) ** 2 - s * s / 4) < 1e-9
    # B_z sits at half-integer x: the same profile shifted by dx/2 moves the centre by dx/2
    B2 = np.zeros_like(E)
    B2[2] = E[1]
    _, b1, _ = M.field_moments(np.zeros_like(E), B2, d)
    assert abs(b1 / m0 - (x0 + d[0] / 2)) < 1e-9
    assert M.field_moments(np.zeros_like(E), B2, d, transverse_only=True)[0] == m0


PINS = [pin_axis_line, pin_accelerating_length, pin_spectrum, pin_beam_moments, pin_field_moments]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_diagnostic_pins(pin):
    pin(D)


def _mutant(tmp_path, name, old, new):
    src = open(os.path.join(HERE, "diagnostics.py")).read()
    assert src.count(old) == 1, old
    f = tmp_path / f"{name}.py"
    f.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"diag_mutant_{name}", f)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MUTANTS = [
    ("no_covariance", pin_beam_moments, "var_p * var_r - cov * cov", "var_p * var_r"),
    ("gamma_not_minus_one", pin_spectrum, "val = u2 / (np.sqrt(1.0 + u2) + 1.0)", "val = np.sqrt(1.0 + u2)"),
    ("bins_off_by_one", pin_spectrum, "ok = (t >= 0) & (idx < nbins)", "ok = (t > 0) & (idx <= nbins - 1)"),
    ("no_stagger", pin_field_moments, "xs = (np.arange(nx) + X_STAGGER[c]) * d[0]", "xs = np.arange(nx) * d[0]"),
    ("y_stagger_swapped", pin_axis_line, "sy, sz = YZ_STAGGER[comp]", "sz, sy = YZ_STAGGER[comp]"),
    ("front_at_sample", pin_accelerating_length, "front = crossing(hi + 1, hi)\n", "front = xs[hi]\n"),
]


@pytest.mark.parametrize("name,pin,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_diagnostic_pin_rejects_planted_mistake(tmp_path, name, pin, old, new):
    with pytest.raises(AssertionError):
        pin(_mutant(tmp_path, name, old, new))
