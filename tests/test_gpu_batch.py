"""Batched launcher: every member of a batch ends bit-identical to the same
setup advanced on its own with pic_step.

The members differ in grid size, solver (perfect dispersion with a moving
window, laser and plasma injection; Yee periodic), current filter, tiling,
guard and sort interval, and each carries two species (a ramped cold plasma
or a uniform warm one, plus a heavier uniform species), so the per-member
sort schedules, window motion, laser planes, loose-particle pass and the
per-species injection tables are all exercised.  The current is summed in
integers, so fields must agree bit for bit; particles are compared by id
(the order inside a cell depends on atomics).
"""
import numpy as np
import pytest

from paper_1204_0838_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import pic  # noqa: E402

D = (0.25, 0.5, 0.5)
STEPS = (17, 23)   # two batch calls
MEMBERS = [
    dict(n=(48, 16, 16), a0=2.0, dens=1.0, tiling=dict(tile=(8, 8, 8), sort_interval=2), jpost="none"),
    dict(n=(40, 24, 16), a0=3.5, dens=1.6, tiling=dict(tile=(8, 4, 4), guard=2, sort_interval=3),
         jpost="binomial"),
    dict(n=(32, 16, 24), a0=4.5, dens=0.7, tiling=dict(tile=(4, 4, 4), guard=0, sort_interval=1), jpost="none"),
    dict(n=(24, 16, 16), yee=True, tiling=dict(tile=(8, 8, 8), interleave=1), jpost="none"),
]
# every member on 8x8x8 tiles with guard 1 (the batch then runs the compiled
# tile body of that shape), ragged grids and different sort schedules
MEMBERS_888 = [
    dict(n=(44, 20, 16), a0=2.5, dens=1.2, tiling=dict(tile=(8, 8, 8), guard=1, sort_interval=2), jpost="none"),
    dict(n=(40, 16, 12), a0=4.0, dens=0.8, tiling=dict(tile=(8, 8, 8), guard=1, sort_interval=3, interleave=4),
         jpost="binomial"),
    dict(n=(20, 12, 16), yee=True, tiling=dict(tile=(8, 8, 8), guard=1, sort_interval=1), jpost="none"),
]


def _make(spec):
    n = spec["n"]
    heavy = inputs.uniform_random_plasma(inputs.Grid(n, D, 0.1), ppc=1, seed=11 + n[0], temperature_ev=2000.0)
    heavy.m = 4.0
    if spec.get("yee"):
        g = inputs.Grid(n, (0.2, 0.2, 0.2), 0.5 * 0.2 / np.sqrt(3.0))
        p = inputs.uniform_random_plasma(g, ppc=4, seed=7, temperature_ev=5000.0, ux_amp=0.05)
        heavy = inputs.uniform_random_plasma(g, ppc=1, seed=8, temperature_ev=2000.0)
        heavy.m = 4.0
        cap = p.count + heavy.count
        sim = pic.Simulation(n, g.d, g.dt, solver="yee", jpost=spec["jpost"], max_particles=cap, **spec["tiling"])
        sim.add_particles(p)
        sim.add_particles(heavy)
        return sim
    cells = n[0] * n[1] * n[2]
    cap0 = cells * 8 + 40 * n[1] * n[2] * 8
    sim = pic.Simulation(n, D, 0.25, solver="pd", bc_x=1, jpost=spec["jpost"], max_particles=cap0 + heavy.count,
                         **spec["tiling"])
    sim.add_empty_species(cap0)
    sim.add_particles(heavy)
    sim.set_plasma(0, x_start=4.0, ramp=8.0, n_plateau=spec["dens"], ppc=(2, 2, 2))
    sim.inject_plasma(0, 0, n[0] - 3)
    sim.set_laser(a0=spec["a0"], omega0=1.508, waist=2.0, fwhm=1.0, t_peak=2.5, t_end=5.0, yc=n[1] * D[1] / 2,
                  zc=n[2] * D[2] / 2, src_x=2)
    sim.set_window(24)
    return sim


def _state(sim):
    out = {"E": sim.E.cpu().numpy(), "B": sim.B.cpu().numpy(), "J": sim.J.cpu().numpy(),
           "window": sim.window_state(), "diag": sim.reduce()}
    for s in range(2):
        p = sim.particles_host(s)
        order = np.argsort(p["id"], kind="stable")
        out[f"p{s}"] = {k: v[..., order] for k, v in p.items()}
    return out


@pytest.mark.parametrize("members", [MEMBERS, MEMBERS_888], ids=["mixed_tilings", "all_8x8x8_guard1"])
def test_batch_members_match_single_runs(members):
    singles = []
    for spec in members:
        sim = _make(spec)
        sim.step(sum(STEPS))
        singles.append(_state(sim))
        sim.close()
    sims = [_make(spec) for spec in members]
    batch = pic.Batch(sims)
    batch.profile_enable(True)
    for k in STEPS:
        batch.step(k)
    batch.sync()
    prof = batch.profile_read()
    assert prof["steps"] == sum(STEPS) and prof["tile_launches"] == 2 * sum(STEPS)
    for i, (sim, ref) in enumerate(zip(sims, singles)):
        got = _state(sim)
        assert got["window"] == ref["window"], i
        if not members[i].get("yee"):
            assert got["window"][0] == sum(STEPS) - 24 + 1          # the window moved
            assert np.abs(ref["E"][1]).max() > 0.1                   # the laser is in
        for f in ("E", "B", "J"):
            assert np.array_equal(got[f], ref[f]), (i, f)
        assert got["diag"]["n_particles"] == ref["diag"]["n_particles"], i
        for s in range(2):
            for k in ("cell", "off", "u", "w", "id"):
                assert np.array_equal(got[f"p{s}"][k], ref[f"p{s}"][k]), (i, s, k)
    batch.close()


def test_batch_rejects_mismatched_members():
    a = _make(MEMBERS[0])
    g = inputs.Grid((16, 16, 16), (0.2, 0.2, 0.2), 0.05)
    b = pic.Simulation(g.n, g.d, g.dt, max_particles=64)
    with pytest.raises(pic.PicError):
        pic.Batch([a, b])          # b has no species
    with pytest.raises(pic.PicError):
        pic.Batch([a, a])          # the same member twice


def test_batch_rejects_denoiser_members():
    g = inputs.Grid((16, 8, 8), (0.2, 0.2, 0.2), 0.05)
    sims = []
    for jpost in ("none", "denoiser"):
        s = pic.Simulation(g.n, g.d, g.dt, jpost=jpost, max_particles=g.ncells)
        s.add_particles(inputs.uniform_random_plasma(g, ppc=1, seed=3))
        sims.append(s)
    b = pic.Batch(sims)
    with pytest.raises(pic.PicError):
        b.step(1)


def test_batch_rest_pass_matches_single_runs():
    """Members whose particles drift beyond their tile's guard between sorts
    (fast beams, guard 0, sort every 4 steps) take the batched rest pass and
    end bit-identical to single runs."""
    def make(n, seed):
        g = inputs.Grid(n, (0.25, 0.3, 0.3), 0.15)
        pl = inputs.uniform_random_plasma(g, ppc=4, seed=seed, temperature_ev=1000.0)
        pl.u[0] += np.float32(2.0)
        sim = pic.Simulation(n, g.d, g.dt, max_particles=pl.count, tile=(4, 4, 4), guard=0, interleave=1,
                             sort_interval=4, threads=256)
        sim.add_particles(pl)
        return sim

    shapes = [((16, 8, 12), 5), ((20, 12, 8), 6)]
    singles = []
    for n, seed in shapes:
        sim = make(n, seed)
        sim.step(9)
        singles.append((sim.E.cpu().numpy(), sim.J.cpu().numpy(), sim.particles_host(0)))
        sim.close()
    sims = [make(n, seed) for n, seed in shapes]
    batch = pic.Batch(sims)
    batch.step(9)
    batch.sync()
    for sim, (E, J, p) in zip(sims, singles):
        assert np.array_equal(sim.E.cpu().numpy(), E) and np.array_equal(sim.J.cpu().numpy(), J)
        q = sim.particles_host(0)
        ia, ib = np.argsort(q["id"]), np.argsort(p["id"])
        for k in ("cell", "off", "u"):
            assert np.array_equal(q[k][..., ia], p[k][..., ib]), k
    batch.close()
