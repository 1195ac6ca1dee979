"""Batched launcher against the FP64 oracle: members of one batch, each a
different setup, advanced together with one launch per phase, are each
checked against the oracle's run of that setup.

Member 0 is the moving-window laser-wakefield run of the single-context
parity test (48x12x12, perfect dispersion at c dt = dx, ramp plasma, laser
through the x boundary, window from step 32, plasma injected at the leading
edge).  Member 1 has another size, laser amplitude, density and tiling and
filters its current binomially.  Member 2 is a periodic Yee grid with a
warm plasma.  Tolerances are the single-context ones: fields and momenta
rel-L2 <= 1e-5 after 48 steps, the same particles (by id).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1204_0838_amd import inputs
from tests.helpers import by_id, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import pic  # noqa: E402

D = (0.25, 0.5, 0.5)
DT = 0.25
STEPS = 48
START = 32
LWFA = [
    dict(n=(48, 12, 12), plasma=dict(x_start=8.0, ramp=10.0, n_plateau=1.0, ppc=(2, 2, 2)),
         laser=dict(a0=2.0, omega0=1.508, waist=1.5, fwhm=1.0, t_peak=4.0, t_end=8.0, yc=3.0, zc=3.0, src_x=2),
         jpost="none", tiling=dict(tile=(8, 8, 8), sort_interval=2)),
    dict(n=(40, 16, 12), plasma=dict(x_start=5.0, ramp=6.0, n_plateau=1.6, ppc=(2, 2, 2)),
         laser=dict(a0=3.5, omega0=1.508, waist=2.0, fwhm=1.0, t_peak=3.0, t_end=7.0, yc=4.0, zc=3.0, src_x=2),
         jpost="binomial", tiling=dict(tile=(8, 4, 4), guard=2, sort_interval=3)),
]
YEE = dict(n=(16, 12, 8), d=(0.2, 0.2, 0.2), ppc=4, seed=21)


def _lwfa_member(spec):
    n = spec["n"]
    cap = n[0] * n[1] * n[2] * 8 + STEPS * n[1] * n[2] * 8
    sim = pic.Simulation(n, D, DT, solver="pd", bc_x=1, jpost=spec["jpost"], max_particles=cap, **spec["tiling"])
    sim.add_empty_species(cap)
    sim.set_plasma(0, **spec["plasma"])
    sim.inject_plasma(0, 0, n[0] - 3)
    sim.set_laser(**spec["laser"])
    sim.set_window(START)
    return sim


def _yee_grid():
    return inputs.Grid(YEE["n"], YEE["d"], 0.5 * YEE["d"][0] / np.sqrt(3.0))


def _yee_member():
    g = _yee_grid()
    pl = inputs.uniform_random_plasma(g, ppc=YEE["ppc"], seed=YEE["seed"], temperature_ev=5000.0, ux_amp=0.05)
    sim = pic.Simulation(g.n, g.d, g.dt, solver="yee", max_particles=pl.count, tile=(8, 4, 4), sort_interval=2)
    sim.add_particles(pl)
    return sim, pl


def _window_particles(sim, n):
    p = sim.particles_host(0)
    _, org = sim.window_state()
    c = p["cell"].astype(np.int64)
    xw = ((c % n[0]) - org) % n[0]
    keep = (c >= 0) & (xw >= 3) & (xw <= n[0] - 4)
    x = np.stack([(xw + p["off"][0]) * D[0], ((c // n[0]) % n[1] + p["off"][1]) * D[1],
                  (c // (n[0] * n[1]) + p["off"][2]) * D[2]])
    return x[:, keep], p["u"][:, keep], p["id"][keep]


def test_batch_members_match_the_oracle():
    print("batch of 3 members vs oracle, 48 steps", flush=True)
    sims = [_lwfa_member(s) for s in LWFA]
    yee, pl = _yee_member()
    sims.append(yee)
    batch = pic.Batch(sims)
    batch.step(20)
    batch.step(STEPS - 20)
    batch.sync()
    for i, spec in enumerate(LWFA):
        g = O.make_grid(spec["n"], D, DT, solver="pd", xbc=1)
        ref = O.run_lwfa(g, O.make_plasma(**spec["plasma"]), O.make_laser(**spec["laser"]), STEPS, START,
                         jpost=1 if spec["jpost"] == "binomial" else 0)
        sim = sims[i]
        assert sim.window_state()[0] == ref["shift"] == STEPS - START + 1
        E, B, _ = sim.fields_window_order()
        assert np.abs(ref["E"][1]).max() > 0.5, i                 # the laser is in
        err = rel_l2(np.concatenate([E, B]), np.concatenate([ref["E"], ref["B"]]))
        print(f"member {i}: field rel-L2 {err:.2e}", flush=True)
        assert err <= 1e-5, i
        x, u, ids = _window_particles(sim, spec["n"])
        assert np.array_equal(np.sort(ids), np.sort(ref["id"])), i
        ug, xg = by_id(ids, u, x)
        uo, xo = by_id(ref["id"], ref["u"], ref["x"])
        assert np.abs(uo).max() > 0.1, i
        assert rel_l2(ug, uo) <= 1e-5, i
        assert np.abs(xg - xo).max() < 1e-5, i
    # the periodic Yee member: 48 oracle steps from the same particles
    g = _yee_grid()
    og = O.from_grid(g)
    x, u, w = pl.positions(g), pl.u.astype(np.float64), pl.w.astype(np.float64)
    E = O.zeros_field(og)
    B = O.zeros_field(og)
    for _ in range(STEPS):
        out = O.step(og, x, u, w, E, B)
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]
    err = rel_l2(np.concatenate([yee.E.cpu().numpy(), yee.B.cpu().numpy()]), np.concatenate([E, B]))
    print(f"member 2 (Yee): field rel-L2 {err:.2e}", flush=True)
    assert err <= 1e-5
    p = yee.particles_host(0)
    assert np.array_equal(np.sort(p["id"]), np.sort(pl.id))
    (ug,) = by_id(p["id"], p["u"])
    (uo,) = by_id(pl.id, u)
    assert rel_l2(ug, uo) <= 1e-5
    batch.close()
