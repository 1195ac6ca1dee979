"""The C2 workload at its full size (Nz = 4096, Nr = 256, 32 particles per
(z, r) cell, 3.3e7 particles), in the launch configuration the benchmark
times (fused tile step, 512-thread tiles, a sort every 16 steps), checked
against the FP64 quasi-cylindrical oracle on sampled outputs:

- after advancing to step 901 (the window has moved since step 800; the
  step taken here includes a window move) one more fused step is taken;
  256 sampled particles (the fastest and random ones) are pushed by the
  oracle from the pre-step state with the pre-step fields: momentum rel-L2
  <= 1e-6, positions within 1e-5 c/w_p;
- the current of that step at 48 sampled (z, r) nodes (where it is largest
  in the bulk and on the axis, and random nodes of the wake region),
  re-deposited by the oracle from every particle that can reach them (their
  pre- and post-step positions as the library stored them): all modes and
  components, rel-L2 <= 1e-5.  (A node's current here sums some 10^3
  contributions of a cold plasma that cancel to a few percent of their
  magnitudes; each FP32 contribution carries ~1e-7 relative error, so the
  sum carries ~1e-7 x (sum of magnitudes / |sum|), measured 2e-6.)"""
import numpy as np
import pytest

from oracle import circ as C
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import workloads  # noqa: E402

STEP = 901


def _window_positions(p, nz, dz, org):
    """FP64 (x, y, z) window positions of (cell, off) with the given origin."""
    c = p["cell"].astype(np.int64)
    iz = c % nz
    izw = (iz - org) % nz
    return np.stack([p["off"][1].astype(np.float64), p["off"][2].astype(np.float64),
                     (izw + p["off"][0].astype(np.float64)) * dz])


def _complex(planes, org):
    a = np.roll(planes.cpu().numpy().astype(np.float64), -org, axis=3)
    return np.ascontiguousarray(np.stack([a[:, 0] + 0j, a[:, 1] + 1j * a[:, 2]]))


def test_c2_full_size_sampled_parity():
    cfg = workloads.C2
    nz, nr, dz, dr, dt = cfg["nz"], cfg["nr"], cfg["dz"], cfg["dr"], cfg["dt"]
    sim = workloads.build_c2(cfg)
    sim.step(STEP)
    sim.sync()
    _, org0 = sim.window_state()
    E0, B0 = _complex(sim.E, org0), _complex(sim.B, org0)
    p0 = sim.particles_host(0)
    sim.step(1)
    sim.sync()
    shift1, org1 = sim.window_state()
    assert org1 == (org0 + 1) % nz                   # this step ends with a window move
    p1 = sim.particles_host(0)
    J = _complex(sim.J, org0)                        # deposited in the pre-move frame

    # live before the step: a valid cell inside window z cells [2, nz - 3]
    c0 = p0["cell"].astype(np.int64)
    izw0 = ((c0 % nz) - org0) % nz
    live = (c0 >= 0) & (izw0 >= 2) & (izw0 <= nz - 3)
    ids0 = p0["id"][live]
    x0 = _window_positions({k: (v[..., live] if isinstance(v, np.ndarray) else v) for k, v in p0.items()},
                           nz, dz, org0)
    u0 = p0["u"][:, live].astype(np.float64)
    w0 = p0["w"][live].astype(np.float64)
    assert len(ids0) > 3e7

    # the same particles after the step (a wall-removed one keeps its arrays, cell -1)
    srt = np.argsort(p1["id"], kind="stable")
    k1 = srt[np.searchsorted(p1["id"][srt], ids0)]
    assert np.array_equal(p1["id"][k1], ids0)
    c1 = p1["cell"][k1].astype(np.int64)
    ok1 = c1 >= 0
    x1 = np.zeros_like(x0)
    x1[0] = p1["off"][1][k1].astype(np.float64)
    x1[1] = p1["off"][2][k1].astype(np.float64)
    x1[2] = (((c1 % nz) - org0) % nz + p1["off"][0][k1].astype(np.float64)) * dz
    u1 = p1["u"][:, k1].astype(np.float64)

    g = C.make_grid(nz, nr, dz, dr, dt)
    rng = np.random.default_rng(2)
    speed = np.sqrt((u0 ** 2).sum(axis=0))
    fast = np.argsort(speed)[-128:]
    rand = rng.choice(len(ids0), 128, replace=False)
    sel = np.unique(np.concatenate([fast, rand]))
    sel = sel[ok1[sel]]
    uo, xo = C.push(g, x0[:, sel], u0[:, sel], E0, B0)
    assert np.abs(uo).max() > 0.1
    assert rel_l2(u1[:, sel], uo) <= 1e-6
    assert np.abs(x1[:, sel] - xo).max() < 1e-5

    # the current at sampled nodes, from every particle that can reach them:
    # the 24 bulk nodes and 8 nodes on or next to the axis where the library's
    # current is largest (the cold plasma elsewhere carries almost none), and
    # 16 random nodes of the region around them
    mag = np.abs(J).sum(axis=(0, 1))                 # [nr, nz]
    mag[:, :40] = 0.0
    mag[:, nz - 40:] = 0.0
    bulk = np.argsort(mag[3:200].ravel())[-24:]
    axis = np.argsort(mag[:2].ravel())[-8:]
    zr = (int(np.argmax(mag.max(axis=0))), 0)
    nodes_z = np.concatenate([bulk % nz, axis % nz, np.clip(zr[0] + rng.integers(-300, 300, 16), 40, nz - 41)])
    nodes_r = np.concatenate([bulk // nz + 3, axis // nz, rng.integers(0, 120, 16)])
    # cells within 4 of a sampled node; a particle is taken if it starts or ends in one
    mask = np.zeros((nr + 8, nz + 8), dtype=bool)
    for iz, jr in zip(nodes_z, nodes_r):
        mask[max(jr - 4, 0):jr + 5, iz - 4:iz + 5] = True
    near = np.zeros(len(ids0), dtype=bool)
    for xx in (x0, x1):
        zc = np.clip(np.floor(xx[2] / dz).astype(np.int64), 0, nz + 7)
        rc = np.clip(np.floor(np.hypot(xx[0], xx[1]) / dr).astype(np.int64), 0, nr + 7)
        near |= mask[rc, zc]
    near &= ok1                                      # (no sampled node lies near the wall)
    assert near.sum() > 10000
    Jo = C.deposit(g, x0[:, near], x1[:, near], u1[:, near], w0[near])
    got = np.array([J[:, :, jr, iz] for iz, jr in zip(nodes_z, nodes_r)])
    want = np.array([Jo[:, :, jr, iz] for iz, jr in zip(nodes_z, nodes_r)])
    assert np.abs(want).max() > 0
    a, b = got.ravel(), want.ravel()
    assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b), np.linalg.norm(a - b) / np.linalg.norm(b)
