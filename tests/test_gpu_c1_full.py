"""Parity at the full C1 size in the launch configuration the benchmark
times (512x256x256 cells, 2.7e8 particles, the cached autotuned tiling, the
fused production step), on outputs the FP64 oracle computes one by one:

- the momentum and position after one step of 256 sampled particles (the
  128 fastest ones, in the wake, and 128 drawn at random), pushed by the
  oracle from the pre-step state and fields;
- the deposited current at 32 sampled cells (16 under fast particles, 16
  random), re-deposited by the oracle from every particle whose stencil can
  reach them.

The run is sampled twice: at step 300, when the laser is in the plasma and
the wake has formed, before the window moves (window origin 0), and at step
520, after the window has moved 35 cells (the storage is then a circular
buffer whose window starts at the origin index; the comparison is made in
window coordinates, in the frame of the step's deposit, before its move).
Tolerances as in the small-grid parity tests: one-step momentum and current
rel-L2 <= 1e-6, positions within 1e-5 cells.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import periodic_delta, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import workloads  # noqa: E402

REACH = 3   # cells: a particle's deposit reaches at most this far from its cell at the step start


def _coords(cell, n, org):
    """Window coordinates of storage cell indices (x counted from the window origin)."""
    return torch.remainder(cell % n[0] - org, n[0]), (cell // n[0]) % n[1], cell // (n[0] * n[1])


def _window_positions(p, n, d, org):
    c = p["cell"].astype(np.int64)
    xw = ((c % n[0]) - org) % n[0]
    idx = (xw, (c // n[0]) % n[1], c // (n[0] * n[1]))
    return np.stack([(idx[a] + p["off"][a].astype(np.float64)) * d[a] for a in range(3)])


def _sampled_step_parity(sim, cfg, seed):
    """One production step of `sim`, checked at sampled particles and cells."""
    n, d = cfg["n"], cfg["d"]
    _, org = sim.window_state()
    v = sim.particles(0)
    cell = v["cell"].long()
    live = cell >= 0
    x, y, z = _coords(cell.clamp(min=0), n, org)
    safe = live & (x >= 8) & (x < n[0] - 8)        # away from the window's kill zones
    u2 = sum(t.double() ** 2 for t in v["u"])
    u2 = torch.where(safe, u2, torch.full_like(u2, -1.0))
    fast = torch.topk(u2, 128).indices
    g = torch.Generator(device="cuda").manual_seed(seed)
    safe_idx = torch.nonzero(safe).squeeze(1)
    rnd = safe_idx[torch.randint(0, safe_idx.numel(), (128,), generator=g, device="cuda")]
    sample = torch.unique(torch.cat([fast, rnd]))
    assert float(u2[fast].min()) > 1e-2             # the fastest sampled particles are relativistic-ish
    # cells where the current is checked (window coordinates)
    pick = torch.cat([fast[:16], rnd[:16]])
    cx, cy, cz = x[pick], y[pick], z[pick]
    near = torch.zeros_like(live)
    for k in range(pick.numel()):
        dx = (x - cx[k]).abs()
        dy = torch.remainder(y - cy[k] + n[1] // 2, n[1]) - n[1] // 2
        dz = torch.remainder(z - cz[k] + n[2] // 2, n[2]) - n[2] // 2
        near |= live & (dx <= REACH) & (dy.abs() <= REACH) & (dz.abs() <= REACH)
    nidx = torch.nonzero(near).squeeze(1)

    def take(idx):
        return {"cell": v["cell"][idx].cpu().numpy(),
                "off": np.stack([t[idx].cpu().numpy() for t in v["off"]]),
                "u": np.stack([t[idx].cpu().numpy() for t in v["u"]]),
                "w": v["w"][idx].cpu().numpy(), "id": v["id"][idx].cpu().numpy()}

    pre_s, pre_n = take(sample), take(nidx)
    E = np.roll(sim.E.cpu().numpy().astype(np.float64), -org, axis=3)
    B = np.roll(sim.B.cpu().numpy().astype(np.float64), -org, axis=3)
    sim.step(1)
    sim.sync()
    v2 = sim.particles(0)
    ids2 = v2["id"].long()
    pos = torch.full((int(ids2.max()) + 1,), -1, dtype=torch.long, device="cuda")
    pos[ids2] = torch.arange(ids2.numel(), device="cuda")

    def after(ids):
        i = pos[torch.as_tensor(ids, dtype=torch.long, device="cuda")]
        assert int(i.min()) >= 0, "a sampled particle was lost"
        return {"cell": v2["cell"][i].cpu().numpy(),
                "off": np.stack([t[i].cpu().numpy() for t in v2["off"]]),
                "u": np.stack([t[i].cpu().numpy() for t in v2["u"]])}

    post_s, post_n = after(pre_s["id"]), after(pre_n["id"])
    # the current of this step was deposited in the frame before the step's window move
    Jg = np.roll(sim.J.cpu().numpy().astype(np.float64), -org, axis=3)

    og = O.make_grid(n, d, cfg["dt"], solver=cfg["solver"], xbc=1)
    L = [n[a] * d[a] for a in range(3)]
    # particles: oracle push from the pre-step state
    x0 = _window_positions(pre_s, n, d, org)
    xw, u1, _ = O.push(og, x0, pre_s["u"].astype(np.float64), E, B)
    assert rel_l2(post_s["u"], u1) <= 1e-6
    xg = _window_positions(post_s, n, d, org)
    err = np.abs(periodic_delta(xg, xw, L)) / np.array(d)[:, None]
    assert err.max() < 1e-5
    # current at the sampled cells from every particle that can reach them
    x0n = _window_positions(pre_n, n, d, org)
    x1n = x0n + periodic_delta(_window_positions(post_n, n, d, org), x0n, L)
    Jo = O.deposit(og, x0n, x1n, pre_n["w"].astype(np.float64), q=-1.0)
    sx, sy, sz = (a.cpu().numpy() for a in (cx, cy, cz))
    got = Jg[:, sz, sy, sx]
    ref = Jo[:, sz, sy, sx]
    assert np.abs(ref).max() > 0
    assert rel_l2(got, ref) <= 1e-6


def test_c1_full_size_sampled_parity():
    cfg = workloads.C1
    start = workloads.window_start_step(cfg)
    sim = workloads.build(cfg)                     # tiling: the autotune cache, as bench.py
    assert start > 301
    print("C1 full size: 300 steps", flush=True)
    sim.step(300)
    sim.sync()
    assert sim.window_state() == (0, 0)
    _sampled_step_parity(sim, cfg, seed=17)
    print(f"C1 full size: to step 520 (window from step {start})", flush=True)
    sim.step(520 - 301)
    sim.sync()
    shift, org = sim.window_state()
    assert shift == 520 - start + 1 and org == shift % cfg["n"][0]
    _sampled_step_parity(sim, cfg, seed=23)
    assert sim.window_state()[0] == shift + 1
    sim.close()
