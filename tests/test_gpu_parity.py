"""GPU parity of the HIP path (called through the C ABI) against the FP64 oracle.

Tolerances: one-step momentum and deposit rel-L2 <= 1e-6 (FP32 arithmetic on
identical FP32 inputs), 16-step field and momentum rel-L2 <= 1e-5, continuity
residual <= 1e-6 max|J|.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1204_0838_amd import inputs
from tests.helpers import absolute_positions, by_id, periodic_delta, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _pic():
    from paper_1204_0838_amd import pic
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return pic


def _sim(grid, max_particles, **kw):
    pic = _pic()
    return pic.Simulation(grid.n, grid.d, grid.dt, solver=grid.solver, bc_x=1 if grid.window else 0,
                          max_particles=max_particles, **kw)


def _set_fields(sim, F6):
    sim.E.copy_(torch.as_tensor(F6[:3]))
    sim.B.copy_(torch.as_tensor(F6[3:]))


RAGGED = inputs.Grid(n=(13, 10, 9), d=(0.3, 0.25, 0.35), dt=0.1)


def _edge_plasma(grid, ppc, seed, temperature_ev):
    """Random plasma plus particles sitting exactly on cell faces and just below them."""
    p = inputs.uniform_random_plasma(grid, ppc=ppc, seed=seed, temperature_ev=temperature_ev, ux_amp=0.05)
    k = min(64, p.count)
    p.off[:, :k // 2] = 0.0
    p.off[:, k // 2:k] = np.float32(1.0) - np.float32(2.0 ** -24)
    return p


@pytest.mark.parametrize("solver", ["yee"])
def test_gather_push_one_step(solver):
    grid = RAGGED
    pl = _edge_plasma(grid, 4, 21, 20000.0)
    F = inputs.random_fields(grid, seed=5, amp=0.5)
    sim = _sim(grid, pl.count)
    sim.add_particles(pl)
    _set_fields(sim, F)
    sim.gather_push(0)
    got = sim.particles_host(0)
    g = O.from_grid(grid)
    x0 = pl.positions(grid)
    xw, u1, x1 = O.push(g, x0, pl.u.astype(np.float64), F[:3].astype(np.float64), F[3:].astype(np.float64))
    assert rel_l2(got["u"], u1) <= 1e-6
    xg = absolute_positions(got["cell"], got["off"], grid.n, grid.d)
    L = [grid.n[a] * grid.d[a] for a in range(3)]
    err = np.abs(periodic_delta(xg, xw, L)) / np.array(grid.d)[:, None]
    assert err.max() < 1e-5   # in cells
    assert np.all(got["off"] >= 0) and np.all(got["off"] < 1)


def test_deposit_parity_and_continuity():
    grid = RAGGED
    pl = _edge_plasma(grid, 4, 22, 50000.0)
    F = inputs.random_fields(grid, seed=6, amp=0.3)
    sim = _sim(grid, pl.count)
    sim.add_particles(pl)
    _set_fields(sim, F)
    sim.gather_push(0)
    sim.deposit(0)
    res, maxj = sim.continuity(0)
    got = sim.particles_host(0)
    Jg = sim.J.cpu().numpy().astype(np.float64)
    assert maxj > 0
    assert res <= 1e-6 * maxj
    g = O.from_grid(grid)
    x0 = pl.positions(grid)
    x1w = absolute_positions(got["cell"], got["off"], grid.n, grid.d)
    L = [grid.n[a] * grid.d[a] for a in range(3)]
    x1 = x0 + periodic_delta(x1w, x0, L)
    Jo = O.deposit(g, x0, x1, pl.w.astype(np.float64), q=-1.0)
    assert rel_l2(Jg, Jo) <= 1e-6
    # independent continuity check: oracle charge densities of the GPU's stored positions
    r0 = O.rho(g, x0, pl.w.astype(np.float64))
    r1 = O.rho(g, x1w, pl.w.astype(np.float64))
    mx, _ = O.continuity(g, r0, r1, Jg)
    assert mx <= 1e-6 * np.abs(Jg).max()


def test_binomial_current_conserves_the_filtered_charge():
    """With the binomial filter the current of the field step is B J; its
    divergence is B div J, so it conserves B rho: pic_continuity filters rho
    once the J planes hold the filtered current (after the field step), and
    not right after the deposit (raw current).  Checked against the oracle's
    residual of the same densities, filtered by the oracle's own filter."""
    grid = RAGGED
    pl = _edge_plasma(grid, 4, 23, 50000.0)
    sim = _sim(grid, pl.count, jpost="binomial")
    sim.add_particles(pl)
    _set_fields(sim, inputs.random_fields(grid, seed=9, amp=0.3))
    sim.gather_push(0)
    sim.deposit(0)
    res_raw, maxj_raw = sim.continuity(0)
    assert maxj_raw > 0 and res_raw <= 1e-6 * maxj_raw
    sim.field_step()
    res, maxj = sim.continuity(0)
    assert res <= 1e-6 * maxj
    got = sim.particles_host(0)
    Jg = sim.J.cpu().numpy().astype(np.float64)
    g = O.from_grid(grid)
    r0 = O.rho(g, pl.positions(grid), pl.w.astype(np.float64))
    r1 = O.rho(g, absolute_positions(got["cell"], got["off"], grid.n, grid.d), pl.w.astype(np.float64))
    f0 = O.binomial(g, np.stack([r0, r0, r0]))[0]
    f1 = O.binomial(g, np.stack([r1, r1, r1]))[0]
    mx, _ = O.continuity(g, f0, f1, Jg)
    assert mx <= 1e-6 * np.abs(Jg).max()
    unfiltered, _ = O.continuity(g, r0, r1, Jg)
    assert unfiltered > 100 * mx                     # the filtered charge is the one it conserves


@pytest.mark.parametrize("solver,window", [("yee", False), ("pd", False), ("pd", True)])
@pytest.mark.parametrize("jpost", ["none", "binomial"])
def test_field_step_parity(solver, window, jpost):
    if solver == "pd":
        grid = inputs.Grid(n=(16, 10, 12), d=(0.25, 0.5, 0.4), dt=0.25, solver="pd", window=window)
    else:
        grid = inputs.Grid(n=(13, 10, 9), d=(0.3, 0.25, 0.35), dt=0.1)
    F = inputs.random_fields(grid, seed=7)
    Jr = inputs.random_fields(grid, seed=8)[:3]
    sim = _pic().Simulation(grid.n, grid.d, grid.dt, solver=solver, bc_x=1 if window else 0, jpost=jpost,
                            max_particles=1)
    _set_fields(sim, F)
    sim.J.copy_(torch.as_tensor(Jr))
    sim.field_step()
    g = O.from_grid(grid)
    J = Jr.astype(np.float64)
    if jpost == "binomial":
        J = O.binomial(g, J)
        assert rel_l2(sim.J.cpu().numpy(), J) <= 1e-6
    E, B = O.field_step(g, F[:3].astype(np.float64), F[3:].astype(np.float64), J)
    assert rel_l2(sim.E.cpu().numpy(), E) <= 1e-6
    assert rel_l2(sim.B.cpu().numpy(), B) <= 1e-6


@pytest.fixture(scope="module")
def c0_oracle():
    grid = inputs.c0_grid()
    pl = inputs.c0_particles(seed=1)
    g = O.from_grid(grid)
    x = pl.positions(grid)
    u = pl.u.astype(np.float64)
    w = pl.w.astype(np.float64)
    E = np.zeros((3, 32, 32, 64))
    B = np.zeros_like(E)
    for _ in range(16):
        out = O.step(g, x, u, w, E, B)
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]
    return {"grid": grid, "particles": pl, "x": x, "u": u, "E": E, "B": B, "J": out["J"]}


def test_c0_sixteen_steps(c0_oracle):
    """64x32x32 periodic, 8 ppc, 10 eV + 0.01c mode, Yee, Courant 0.5, 16 steps."""
    grid, pl = c0_oracle["grid"], c0_oracle["particles"]
    sim = _sim(grid, pl.count)
    sim.add_particles(pl)
    sim.step(15)
    sim.gather_push(0)
    sim.deposit(0)
    res, maxj = sim.continuity(0)
    sim.field_step()
    got = sim.particles_host(0)
    assert res <= 1e-6 * maxj
    F_gpu = np.concatenate([sim.E.cpu().numpy(), sim.B.cpu().numpy()])
    F_ora = np.concatenate([c0_oracle["E"], c0_oracle["B"]])
    assert rel_l2(F_gpu, F_ora) <= 1e-5
    assert rel_l2(sim.E.cpu().numpy(), c0_oracle["E"]) <= 1e-5
    assert rel_l2(sim.J.cpu().numpy(), c0_oracle["J"]) <= 1e-5
    ug, = by_id(got["id"], got["u"])
    assert rel_l2(ug, c0_oracle["u"]) <= 1e-5
    xg = absolute_positions(got["cell"], got["off"], grid.n, grid.d)
    xg, = by_id(got["id"], xg)
    L = [grid.n[a] * grid.d[a] for a in range(3)]
    assert np.abs(periodic_delta(xg, c0_oracle["x"], L)).max() < 1e-5
    d = sim.reduce()
    dv = 0.2 ** 3
    assert d["n_particles"] == pl.count
    assert abs(d["charge"] - (-1.0) * pl.w.astype(np.float64).sum() * dv) < 1e-9 * pl.count * dv
    od = O.diag(O.from_grid(grid), c0_oracle["u"], pl.w, c0_oracle["E"], c0_oracle["B"])
    assert abs(d["e_kin"] / od["e_kin"] - 1) < 1e-5
    assert abs(d["e_field"] / od["e_field"] - 1) < 1e-4


def test_step_equals_split_path_bit_exact():
    grid = RAGGED
    pl = inputs.uniform_random_plasma(grid, ppc=4, seed=31, temperature_ev=5000.0, ux_amp=0.05)
    a = _sim(grid, pl.count)
    b = _sim(grid, pl.count)
    a.add_particles(pl)
    b.add_particles(pl)
    a.step(5)
    for _ in range(5):
        b.gather_push(0)
        b.deposit(0)
        b.field_step()
    for fa, fb in ((a.E, b.E), (a.B, b.B), (a.J, b.J)):
        assert torch.equal(fa, fb)
    pa, pb = a.particles_host(0), b.particles_host(0)
    ia, ib = np.argsort(pa["id"]), np.argsort(pb["id"])
    assert np.array_equal(pa["u"][:, ia], pb["u"][:, ib])
    assert np.array_equal(pa["off"][:, ia], pb["off"][:, ib])
    assert np.array_equal(pa["cell"][ia], pb["cell"][ib])


def test_empty_species_is_vacuum_evolution():
    grid = inputs.Grid(n=(16, 8, 8), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    sim = _sim(grid, 16)
    sim.add_species(np.zeros(0, np.int32), np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32),
                    np.zeros(0, np.float32), np.zeros(0, np.int32), capacity=16)
    F = inputs.random_fields(grid, seed=9)
    _set_fields(sim, F)
    sim.step(3)
    g = O.from_grid(grid)
    E, B = F[:3].astype(np.float64), F[3:].astype(np.float64)
    for _ in range(3):
        E, B = O.field_step(g, E, B)
    assert rel_l2(sim.E.cpu().numpy(), E) <= 1e-6
    assert sim.reduce()["n_particles"] == 0


def test_light_speed_step_at_the_courant_limit_is_reported():
    """Perfect dispersion at c dt = dx: a particle with u_x = 1e8 has v_x = 1
    in FP32 (sqrt(1 + u^2) rounds to u), a move of exactly one cell, which the
    deposit's support does not cover: PIC_ECFL at the next sync."""
    pic = _pic()
    grid = inputs.Grid(n=(16, 8, 8), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    pl = inputs.uniform_random_plasma(grid, ppc=1, seed=4)
    pl.u[:] = 0.0
    pl.u[0, 3] = 1e8
    sim = _sim(grid, pl.count)
    sim.add_particles(pl)
    sim.gather_push(0)
    with pytest.raises(pic.PicError) as e:
        sim.sync()
    assert e.value.status == pic.PIC_ECFL


def test_injection_beyond_capacity_is_refused():
    """Plasma injection that could exceed the species' capacity is refused on
    the host before any launch (the host keeps an upper bound of the live
    count, re-read from the device when it gets close): PIC_ENOMEM, and a
    slab that fits is then injected in full."""
    pic = _pic()
    grid = inputs.Grid(n=(16, 8, 8), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    sim = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", bc_x=1, max_particles=1024)
    sim.add_empty_species(1024)
    sim.set_plasma(0, x_start=0.0, ramp=0.0, n_plateau=1.0, ppc=(2, 2, 2))
    with pytest.raises(pic.PicError) as e:
        sim.inject_plasma(0, 4, 7)   # up to 3 x 8 x 8 cells at 8 per cell = 1536 > 1024
    assert e.value.status == pic.PIC_ENOMEM
    sim2 = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", bc_x=1, max_particles=1024)
    sim2.add_empty_species(1024)
    sim2.set_plasma(0, x_start=0.0, ramp=0.0, n_plateau=1.0, ppc=(2, 2, 2))
    sim2.inject_plasma(0, 4, 6)      # 2 x 8 x 8 cells at 8 per cell = 1024: exactly the capacity
    # (window cells 4 and 5: the first three are the window's removal margin)
    sim2.sync()
    assert sim2.reduce()["n_particles"] == 1024


def test_non_finite_momentum_is_reported():
    pic = _pic()
    grid = RAGGED
    pl = inputs.uniform_random_plasma(grid, ppc=1, seed=3)
    pl.u[0, 5] = np.nan
    sim = _sim(grid, pl.count)
    sim.add_particles(pl)
    sim.gather_push(0)
    with pytest.raises(pic.PicError) as e:
        sim.sync()
    assert e.value.status == pic.PIC_ENONFINITE
