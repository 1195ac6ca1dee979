"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test fixes a property that the mathematics (or the paper) determines
independently of the oracle's code, chosen so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails at least one.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1204_0838_amd import inputs


# ---------------------------------------------------------------- shape
def test_spline_partition_of_unity_moment_and_positivity():
    rng = np.random.default_rng(0)
    for s in rng.uniform(-5, 5, 200):
        i = math.floor(s)
        nodes = np.arange(i - 3, i + 5)
        w = np.array([O.bspline3(n - s) for n in nodes])
        assert np.all(w >= 0)
        assert abs(w.sum() - 1.0) < 1e-15
        assert abs((nodes * w).sum() - s) < 1e-13          # reproduces linears
        # second moment of the cubic B-spline: variance 4/12 = 1/3
        assert abs(((nodes - s) ** 2 * w).sum() - 1.0 / 3.0) < 1e-13
        assert np.count_nonzero(w) <= 4


def test_spline_closed_form_node_weights_and_c2():
    # weights on nodes i-1..i+2 for offset delta: (1-d)^3/6, (4-6d^2+3d^3)/6, (1+3d+3d^2-3d^3)/6, d^3/6
    for d in np.linspace(0, 1, 11, endpoint=False):
        ref = [(1 - d) ** 3 / 6, (4 - 6 * d * d + 3 * d ** 3) / 6, (1 + 3 * d + 3 * d * d - 3 * d ** 3) / 6, d ** 3 / 6]
        got = [O.bspline3(m - d) for m in (-1, 0, 1, 2)]
        assert np.allclose(got, ref, atol=1e-15, rtol=0)
    # C2 continuity at the knots |xi| = 1, 2 (finite differences of value, slope, curvature)
    h = 1e-5
    for knot in (1.0, 2.0, -1.0, -2.0, 0.0):
        f = [O.bspline3(knot + k * h) for k in (-2, -1, 0, 1, 2)]
        d1l, d1r = (f[2] - f[1]) / h, (f[3] - f[2]) / h
        assert abs(d1l - d1r) < 1e-4
        c_l, c_r = (f[2] - 2 * f[1] + f[0]) / h ** 2, (f[4] - 2 * f[3] + f[2]) / h ** 2
        assert abs(c_l - c_r) < 1e-3
    # unit integral
    xs = np.linspace(-2, 2, 40001)
    vals = np.array([O.bspline3(x) for x in xs])
    assert abs(np.trapezoid(vals, xs) - 1.0) < 1e-8


# ---------------------------------------------------------------- gather
def _grid(n=(8, 6, 5), d=(0.3, 0.25, 0.4), dt=0.05):
    return O.make_grid(n, d, dt)


def _staggered_coords(g, sh):
    n = [int(g.n[a]) for a in range(3)]
    ax = [(np.arange(n[a]) + sh[a]) * g.d[a] for a in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return x, y, z


STAG_E = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5)]
STAG_B = [(0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]


def test_gather_constant_and_linear_fields_exact():
    g = _grid()
    n = [int(g.n[a]) for a in range(3)]
    L = [n[a] * g.d[a] for a in range(3)]
    rng = np.random.default_rng(1)
    E = np.zeros((3, n[2], n[1], n[0]))
    B = np.zeros_like(E)
    consts = rng.normal(size=6)
    for c in range(3):
        E[c] = consts[c]
        B[c] = consts[3 + c]
    for _ in range(20):
        x = rng.uniform(0, 1, 3) * L
        ep, bp = O.gather(g, E, B, x)
        assert np.allclose(np.r_[ep, bp], consts, atol=1e-14, rtol=0)
    # linear field in y and z for every component, on a bounded-x grid far from the edges
    # (periodic axes cannot hold a linear field, so test away from the wrap along y/z)
    gb = O.make_grid((12, 12, 12), (0.3, 0.25, 0.4), 0.05, xbc=1)
    n = [12, 12, 12]
    slopes = rng.normal(size=(6, 3))
    E = np.zeros((3, 12, 12, 12))
    B = np.zeros_like(E)
    for c in range(3):
        x, y, z = _staggered_coords(gb, STAG_E[c])
        E[c] = 1.0 + slopes[c, 0] * x + slopes[c, 1] * y + slopes[c, 2] * z
        x, y, z = _staggered_coords(gb, STAG_B[c])
        B[c] = -2.0 + slopes[3 + c, 0] * x + slopes[3 + c, 1] * y + slopes[3 + c, 2] * z
    for _ in range(20):
        p = np.array([rng.uniform(4, 7) * 0.3, rng.uniform(4, 7) * 0.25, rng.uniform(4, 7) * 0.4])
        ep, bp = O.gather(gb, E, B, p)
        want_e = [1.0 + slopes[c] @ p for c in range(3)]
        want_b = [-2.0 + slopes[3 + c] @ p for c in range(3)]
        assert np.allclose(ep, want_e, atol=1e-12, rtol=0)
        assert np.allclose(bp, want_b, atol=1e-12, rtol=0)


def test_gather_brute_force_against_continuous_shape_sum():
    """Gather equals sum over all grid points of F * S((X - x)/d) per axis (brute force, periodic images)."""
    g = _grid(n=(6, 5, 5))
    n = [int(g.n[a]) for a in range(3)]
    rng = np.random.default_rng(2)
    E = rng.normal(size=(3, n[2], n[1], n[0]))
    B = rng.normal(size=(3, n[2], n[1], n[0]))
    x = rng.uniform(0, 1, 3) * np.array([n[a] * g.d[a] for a in range(3)])
    ep, bp = O.gather(g, E, B, x)

    def brute(F, sh):
        tot = 0.0
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    wgt = 1.0
                    for a, idx in enumerate((i, j, k)):
                        L = n[a]
                        s = x[a] / g.d[a] - sh[a]
                        wgt *= sum(O.bspline3(idx + img * L - s) for img in (-1, 0, 1))
                    tot += F[k, j, i] * wgt
        return tot

    assert np.allclose(ep, [brute(E[c], STAG_E[c]) for c in range(3)], atol=1e-12)
    assert np.allclose(bp, [brute(B[c], STAG_B[c]) for c in range(3)], atol=1e-12)


# ---------------------------------------------------------------- Boris
def test_boris_gyration_closed_form():
    Bz, dt, qm = 1.3, 0.2, -1.0
    u = np.array([0.5, 0.0, 0.2])
    gam = math.sqrt(1 + u @ u)
    theta = 2 * math.atan(abs(qm) * Bz * dt / (2 * gam))
    uu = u.copy()
    for n in range(1, 1001):
        uu = O.boris(uu, [0, 0, 0], [0, 0, Bz], qm, dt)
        if n in (1, 17, 1000):
            ang = math.atan2(uu[1], uu[0])
            want = math.remainder(n * theta, 2 * math.pi)   # electron in +B_z rotates counter-clockwise
            assert abs(math.remainder(ang - want, 2 * math.pi)) < 1e-11
    assert abs(np.linalg.norm(uu) - np.linalg.norm(u)) < 1e-14
    assert uu[2] == u[2]


def test_boris_uniform_electric_field_exact():
    E = np.array([0.3, -0.2, 0.05])
    u = np.array([0.1, 0.0, -0.4])
    dt, qm = 0.05, -1.0
    uu = u.copy()
    for _ in range(400):
        uu = O.boris(uu, E, [0, 0, 0], qm, dt)
    assert np.allclose(uu, u + qm * E * 400 * dt, atol=1e-13, rtol=0)


def test_boris_exb_drift():
    # E along x, B along z: drift velocity E x B / B^2 = (0, -E/B, 0)
    E0, B0, qm = 1e-4, 1.0, -1.0
    nper = 64
    dt = 2 * math.tan(math.pi / nper) / (abs(qm) * B0)   # exactly 64 steps per gyration
    u = np.zeros(3)
    x = np.zeros(3)
    steps = nper * 20
    for _ in range(steps):
        u = O.boris(u, [E0, 0, 0], [0, 0, B0], qm, dt)
        x += dt * u / math.sqrt(1 + u @ u)
    v = x / (steps * dt)
    assert abs(v[1] - (-E0 / B0)) < 1e-6 * (E0 / B0)
    assert abs(v[0]) < 1e-6 * (E0 / B0)
    # the drift velocity is a fixed point of the rotation up to the O(v^2) gamma correction
    ud = np.array([0.0, -E0 / B0, 0.0])
    ud2 = O.boris(ud, [E0, 0, 0], [0, 0, B0], qm, dt)
    assert np.allclose(ud2, ud, atol=1e-8 * E0, rtol=0)   # gamma - 1 ~ 5e-9 here


# ---------------------------------------------------------------- deposit
def _random_moves(g, npart, rng, max_cells=0.95):
    n = np.array([int(g.n[a]) for a in range(3)])
    d = np.array([g.d[a] for a in range(3)])
    x0 = rng.uniform(0, 1, (3, npart)) * (n * d)[:, None]
    step = rng.uniform(-max_cells, max_cells, (3, npart)) * d[:, None]
    return x0, x0 + step


@pytest.mark.parametrize("xbc", [0, 1])
def test_deposit_continuity_to_roundoff(xbc):
    g = O.make_grid((10, 7, 6), (0.25, 0.4, 0.35), 0.1, xbc=xbc)
    rng = np.random.default_rng(3)
    x0, x1 = _random_moves(g, 300, rng)
    if xbc == 1:   # keep supports inside the bounded x range
        x0[0] = rng.uniform(3, 7, 300) * 0.25
        x1[0] = x0[0] + rng.uniform(-0.95, 0.95, 300) * 0.25
    w = rng.uniform(0.05, 0.2, 300)
    J = O.deposit(g, x0, x1, w, q=-1.0)
    x1w = x1.copy()
    if xbc == 0:
        L = np.array([int(g.n[a]) * g.d[a] for a in range(3)])
        x1w = x1 - L[:, None] * np.floor(x1 / L[:, None])
    else:
        for a in (1, 2):
            L = int(g.n[a]) * g.d[a]
            x1w[a] = x1[a] - L * np.floor(x1[a] / L)
    r0 = O.rho(g, x0, w)
    r1 = O.rho(g, x1w, w)
    mx, _ = O.continuity(g, r0, r1, J)
    assert np.abs(J).max() > 0
    assert mx <= 1e-13 * np.abs(J).max()


def test_deposit_current_sum_rule_and_rest():
    g = _grid(n=(9, 8, 7))
    rng = np.random.default_rng(4)
    x0, x1 = _random_moves(g, 50, rng)
    w = rng.uniform(0.1, 0.3, 50)
    q = -1.0
    J = O.deposit(g, x0, x1, w, q=q)
    # sum over nodes of J_d equals sum_p q w (x1 - x0)_d / dt  (first-moment identity of the spline)
    want = (q * w[None, :] * (x1 - x0)).sum(axis=1) / g.dt
    got = J.reshape(3, -1).sum(axis=1)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-13)
    # a particle at rest deposits nothing
    J0 = O.deposit(g, x0, x0, w, q=q)
    assert np.abs(J0).max() == 0.0


def test_deposit_single_particle_brute_force_1d_motion():
    """Motion along x only: the current through face i+1/2 is minus the change of the
    charge on the nodes left of it per step, J_x(i+1/2) = -(dx/dt) q w (Q_left1 - Q_left0) S_y S_z."""
    g = _grid(n=(10, 8, 8))
    q, w = -1.0, 0.125
    x0 = np.array([[1.37], [0.91], [1.22]])
    x1 = x0 + np.array([[0.2], [0.0], [0.0]])
    J = O.deposit(g, x0, x1, np.array([w]), q=q)
    nx, ny, nz = 10, 8, 8
    want = np.zeros((nz, ny, nx))
    sx0, sx1 = x0[0, 0] / g.d[0], x1[0, 0] / g.d[0]
    for i in range(nx):
        left0 = sum(O.bspline3(m - sx0) for m in range(-5, i + 1))
        left1 = sum(O.bspline3(m - sx1) for m in range(-5, i + 1))
        for j in range(ny):
            for k in range(nz):
                wy = O.bspline3(j - x0[1, 0] / g.d[1])
                wz = O.bspline3(k - x0[2, 0] / g.d[2])
                want[k, j, i] = -(g.d[0] / g.dt) * q * w * (left1 - left0) * wy * wz
    assert np.abs(want).max() > 0.01
    assert np.allclose(J[0], want, atol=1e-13)
    assert np.abs(J[1]).max() < 1e-15 and np.abs(J[2]).max() < 1e-15


# ---------------------------------------------------------------- field solvers
def _mode_field(g, comp, k):
    n = [int(g.n[a]) for a in range(3)]
    E = np.zeros((3, n[2], n[1], n[0]))
    x, y, z = _staggered_coords(g, STAG_E[comp])
    E[comp] = np.cos(k[0] * x + k[1] * y + k[2] * z)
    return E


def _symbol(g, axis, k):
    """Fourier symbol of the transverse smoothing S_axis (stencil of Section 2)."""
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    c1, c2 = math.cos(k[t1] * g.d[t1]), math.cos(k[t2] * g.d[t2])
    return g.alpha[axis] + 2 * g.beta[t1] * c1 + 2 * g.beta[t2] * c2 + 4 * g.gam[axis] * c1 * c2


def _theta(g, k, comp):
    lam = 0.0
    for a in range(3):
        if a == comp:
            continue
        s = math.sin(k[a] * g.d[a] / 2) ** 2
        lam += _symbol(g, a, k) * (2 / g.d[a]) ** 2 * s
    return 2 * math.asin(g.dt * math.sqrt(lam) / 2)


@pytest.mark.parametrize("solver", ["yee", "pd"])
@pytest.mark.parametrize("comp,mvec", [(1, (3, 0, 2)), (2, (1, 2, 0)), (0, (0, 1, 3))])
def test_vacuum_eigenmode_dispersion(solver, comp, mvec):
    n, d = (16, 8, 8), (0.25, 0.5, 0.4)
    dt = 0.25 if solver == "pd" else 0.9 / math.sqrt(sum(1 / di ** 2 for di in d))
    g = O.make_grid(n, d, dt, solver=solver)
    k = [2 * math.pi * mvec[a] / (n[a] * d[a]) for a in range(3)]
    E0 = _mode_field(g, comp, k)
    B = np.zeros_like(E0)
    E = E0.copy()
    th = _theta(g, k, comp)
    for step in range(1, 41):
        E, B = O.field_step(g, E, B)
    assert np.allclose(E, E0 * math.cos(40 * th), atol=1e-11)


def test_pd_on_axis_has_no_numerical_dispersion():
    n, d = (32, 4, 4), (0.25, 0.5, 0.5)
    g = O.make_grid(n, d, 0.25, solver="pd")
    for m in (1, 5, 11, 15):
        k = 2 * math.pi * m / (n[0] * d[0])
        E0 = _mode_field(g, 1, (k, 0, 0))
        E, B = E0.copy(), np.zeros_like(E0)
        for _ in range(25):
            E, B = O.field_step(g, E, B)
        # omega = c k exactly: phase advance k dx per step
        assert np.allclose(E, E0 * math.cos(25 * k * d[0]), atol=1e-11)


def _pd_vertex_values(alpha, beta, gam, d, dt):
    vals = []
    for sx in (0, 1):
        for sy in (0, 1):
            for sz in (0, 1):
                s = (sx, sy, sz)
                f = 0.0
                for a in range(3):
                    t1, t2 = (a + 1) % 3, (a + 2) % 3
                    c1, c2 = 1 - 2 * s[t1], 1 - 2 * s[t2]
                    sig = alpha[a] + 2 * beta[t1] * c1 + 2 * beta[t2] * c2 + 4 * gam[a] * c1 * c2
                    f += sig * (dt / d[a]) ** 2 * s[a]
                vals.append(f)
    return np.array(vals)


@pytest.mark.parametrize("ratio", [1.0, 0.75, 0.5, 0.12])
def test_pd_stability_vertices_and_bounded_noise_run(ratio):
    """With c dt = dx every vertex of the symbol cube lies in [0, 1] iff dx <= dy, dz.

    The on-axis Nyquist mode sits exactly on the boundary (phase advance pi per
    step), where the leapfrog has a double eigenvalue -1: raw noise there grows
    linearly, never exponentially.  Noise without Nyquist content stays bounded.
    """
    d = (0.25, 0.25 / ratio, 0.25 / ratio)
    a, b, gm = O.pd_coeffs(d)
    v = _pd_vertex_values(a, b, gm, d, d[0])
    assert v.min() >= -1e-15 and v.max() <= 1 + 1e-15
    g = O.make_grid((12, 6, 6), d, d[0], solver="pd")
    rng = np.random.default_rng(5)
    E0 = rng.uniform(-1, 1, (3, 6, 6, 12))
    B0 = rng.uniform(-1, 1, (3, 6, 6, 12))
    E, B = O.binomial(g, E0), O.binomial(g, B0)       # removes every Nyquist component
    m0 = max(np.abs(E).max(), np.abs(B).max())
    for _ in range(900):
        E, B = O.field_step(g, E, B)
    assert max(np.abs(E).max(), np.abs(B).max()) < 2 * m0
    E, B = E0.copy(), B0.copy()
    amp = []
    for s in range(1, 601):
        E, B = O.field_step(g, E, B)
        if s in (150, 300, 600):
            amp.append(np.abs(E).max())
    assert amp[2] / amp[1] < 2.3 and amp[1] / amp[0] < 2.3   # at most linear growth
    assert np.abs(B).max() < 3 * np.abs(B0).max()


def test_identity_stencil_at_dt_equal_dx_is_unstable():
    """Negative control: plain Yee (S = identity) at c dt = dx in 3D violates the Courant limit."""
    d = (0.25, 0.25, 0.25)
    g = O.make_grid((8, 8, 8), d, 0.25, solver="yee")
    rng = np.random.default_rng(6)
    E = rng.uniform(-1, 1, (3, 8, 8, 8))
    B = np.zeros_like(E)
    for _ in range(200):
        E, B = O.field_step(g, E, B)
    assert np.abs(E).max() > 1e3


def test_pd_requires_coarse_longitudinal_axis():
    with pytest.raises(ValueError):
        O.pd_coeffs((0.5, 0.25, 0.5))
    # manual coefficients of the same form with dx > dy: a vertex exceeds 1 (unstable)
    d = (0.5, 0.4, 0.5)
    ry, rz = (d[0] / d[1]) ** 2, (d[0] / d[2]) ** 2
    beta = np.array([1 / 8, ry / 8, rz / 8])
    gam = np.array([ry * rz / 16, rz / 16, ry / 16])
    alpha = np.array([1 - 2 * beta[(a + 1) % 3] - 2 * beta[(a + 2) % 3] - 4 * gam[a] for a in range(3)])
    assert _pd_vertex_values(alpha, beta, gam, d, d[0]).max() > 1.0


def test_yee_preserves_div_b_and_pd_stencil_reduces_to_identity():
    g = O.make_grid((8, 6, 6), (0.3, 0.3, 0.3), 0.1)
    rng = np.random.default_rng(7)
    E = rng.normal(size=(3, 6, 6, 8))
    B = np.zeros_like(E)
    J = rng.normal(size=E.shape)
    for _ in range(5):
        E, B = O.field_step(g, E, B, J)
    assert np.abs(O.div_b(g, B)).max() < 1e-11
    a, b, gm = O.pd_coeffs((0.3, 0.3, 0.3), variant=2)
    assert np.all(a == 1) and np.all(b == 0) and np.all(gm == 0)


@pytest.mark.parametrize("solver", ["yee", "pd"])
def test_gauss_law_residual_constant_in_full_pic_cycle(solver):
    n, d = (12, 6, 6), (0.2, 0.3, 0.3)
    dt = 0.2 if solver == "pd" else 0.5 * 0.2 / math.sqrt(3)
    grid = inputs.Grid(n=n, d=d, dt=dt, solver=solver)
    g = O.from_grid(grid)
    pl = inputs.uniform_random_plasma(grid, ppc=4, seed=11, temperature_ev=2000.0, ux_amp=0.05)
    x = pl.positions(grid)
    u = pl.u.astype(np.float64)
    w = pl.w.astype(np.float64)
    E = np.zeros((3, n[2], n[1], n[0]))
    B = np.zeros_like(E)
    r0 = O.rho(g, x, w)
    for _ in range(6):
        out = O.step(g, x, u, w, E, B)
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]
    r1 = O.rho(g, x, w)
    diff = O.div_e(g, E) - (r1 - r0)
    assert np.abs(diff).max() < 1e-11 * max(1.0, np.abs(r0).max())


# ---------------------------------------------------------------- filter
def test_binomial_transfer_function_and_dc_gain():
    n, d = (16, 8, 8), (0.25, 0.5, 0.5)
    g = O.make_grid(n, d, 0.1)
    m = (3, 2, 1)
    k = [2 * math.pi * m[a] / (n[a] * d[a]) for a in range(3)]
    J = np.zeros((3, 8, 8, 16))
    for c in range(3):
        x, y, z = _staggered_coords(g, STAG_E[c])
        J[c] = np.cos(k[0] * x + k[1] * y + k[2] * z)
    out = O.binomial(g, J)
    gain = np.prod([math.cos(k[a] * d[a] / 2) ** 2 for a in range(3)])
    assert np.allclose(out, gain * J, atol=1e-13)
    const = np.full_like(J, 2.5)
    assert np.allclose(O.binomial(g, const), const, atol=1e-15)


# ---------------------------------------------------------------- whole cycle
def test_langmuir_frequency_quiet_start():
    """Cold quiet-start plasma mode k = 2 pi / Lx on the 0.2 c/w_p grid.

    Linear theory for momentum-conserving cubic gather + charge-conserving
    cubic deposit + leapfrog: w^2 = w_p^2 (k/K) Shat^2 with K = k sinc(k dx/2),
    Shat = sinc^4(k dx / 2), then sin(w dt/2) = (dt/2) w_c.
    """
    n, d = (64, 4, 4), (0.2, 0.2, 0.2)
    dt = 0.5 * 0.2 / math.sqrt(3)
    grid = inputs.Grid(n=n, d=d, dt=dt)
    g = O.from_grid(grid)
    pl = inputs.lattice_plasma(grid, (2, 2, 2), ux_amp=1e-5)
    x = pl.positions(grid)
    u = pl.u.astype(np.float64)
    w = pl.w.astype(np.float64)
    E = np.zeros((3, n[2], n[1], n[0]))
    B = np.zeros_like(E)
    xs = (np.arange(n[0]) + 0.5) * d[0]
    kx = 2 * math.pi / (n[0] * d[0])
    amp = []
    for _ in range(240):
        out = O.step(g, x, u, w, E, B)
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]
        amp.append((E[0].mean(axis=(0, 1)) * np.exp(1j * kx * xs)).sum())
    a = np.array(amp)
    a = a.real if np.abs(a.real).max() > np.abs(a.imag).max() else a.imag
    cos_th = (a[1:-1] * (a[2:] + a[:-2])).sum() / (2 * (a[1:-1] ** 2).sum())
    omega = math.acos(cos_th) / dt
    h = kx * d[0] / 2
    wc = math.sqrt((math.sin(h) / h) ** 7)
    want = 2 / dt * math.asin(dt / 2 * wc)
    assert abs(want - 0.998734) < 2e-6
    assert abs(omega / want - 1) < 1e-5


def test_oracle_reports_non_finite_input():
    grid = inputs.Grid(n=(8, 4, 4), d=(0.2, 0.2, 0.2), dt=0.05)
    g = O.from_grid(grid)
    pl = inputs.uniform_random_plasma(grid, ppc=1, seed=3)
    x = pl.positions(grid)
    u = pl.u.astype(np.float64)
    u[0, 3] = np.nan
    E = np.zeros((3, 4, 4, 8))
    with pytest.raises(FloatingPointError):
        O.step(g, x, u, pl.w.astype(np.float64), E, E.copy())
