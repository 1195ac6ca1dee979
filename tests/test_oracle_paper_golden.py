"""Checks tied to numbers the paper prints (fixtures in tests/golden/, each cited)."""
import json
import math
import os

import numpy as np

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_run_parameters.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def test_plasma_frequency_normalisation_matches_printed_gamma_g():
    """Section 1 defines w_pe = (n0 e^2 / m_e eps0)^(1/2); Section 3.1 prints
    gamma_g = w0/w_pe ~ 16.3 for lambda0 = 0.805 um, n0 = 6.5e18 cm^-3."""
    g = _gold()
    e, me, eps0, c = 1.602176634e-19, 9.1093837015e-31, 8.8541878128e-12, 299792458.0
    n0 = g["plateau_density_cm3"] * 1e6
    wpe = math.sqrt(n0 * e * e / (me * eps0))
    w0 = 2 * math.pi * c / (g["laser_wavelength_um"] * 1e-6)
    assert abs(w0 / wpe - g["gamma_g_printed"]) < 0.05
    # printed grid spacings agree with the printed fractions of lambda0
    assert abs(g["vorpal_pd_dx_over_lambda0"] * 805 - g["vorpal_pd_dx_nm"]) < 0.1
    assert abs(g["vorpal_pd_dy_over_lambda0"] * 805 - g["vorpal_pd_dy_nm"]) < 0.6


def test_pd_stencil_at_the_papers_aspect_ratio():
    """The paper's grid (dx = 0.06 lambda0, dy = dz = 0.5 lambda0) meets its stated
    constraint dx <= dy, dz; at c dt = dx the oracle's stencil then propagates
    on-axis waves without dispersion and keeps every symbol vertex in [0, 1]."""
    g = _gold()
    ratio = g["vorpal_pd_dx_over_lambda0"] / g["vorpal_pd_dy_over_lambda0"]
    d = (1.0, 1.0 / ratio, 1.0 / ratio)
    a, b, gm = O.pd_coeffs(d)
    for sx in (0, 1):
        for sy in (0, 1):
            for sz in (0, 1):
                s = (sx, sy, sz)
                f = 0.0
                for ax in range(3):
                    t1, t2 = (ax + 1) % 3, (ax + 2) % 3
                    c1, c2 = 1 - 2 * s[t1], 1 - 2 * s[t2]
                    sig = a[ax] + 2 * b[t1] * c1 + 2 * b[t2] * c2 + 4 * gm[ax] * c1 * c2
                    f += sig * (d[0] / d[ax]) ** 2 * s[ax]
                assert -1e-15 <= f <= 1 + 1e-15
    n = (24, 4, 4)
    grid = O.make_grid(n, d, d[0], solver="pd")
    k = 2 * math.pi * 5 / (n[0] * d[0])
    x = (np.arange(n[0])) * d[0]
    E0 = np.zeros((3, 4, 4, 24))
    E0[1] = np.cos(k * x)[None, None, :]
    E, B = E0.copy(), np.zeros_like(E0)
    for _ in range(30):
        E, B = O.field_step(grid, E, B)
    assert np.allclose(E, E0 * math.cos(30 * k * d[0]), atol=1e-11)
