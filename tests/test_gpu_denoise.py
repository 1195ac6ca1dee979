"""GPU parity of the learned current denoiser (bf16 matrix-core convolutions)
against the FP64 oracle that mirrors its bf16 roundings, on periodic and
moving-window grids whose sizes leave ragged tiles on every axis."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import pic  # noqa: E402


def _bf16_array(a):
    return np.vectorize(O.bf16)(np.asarray(a, dtype=np.float64))


def _params(seed, H=32):
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, 3, 3, 3, 3)) / np.sqrt(81.0)
    W2 = rng.standard_normal((H, H, 3, 3, 3)) / np.sqrt(27.0 * H)
    W3 = 0.5 * rng.standard_normal((3, H, 3, 3, 3)) / np.sqrt(27.0 * H)
    b1 = 0.1 * rng.standard_normal(H)
    b2 = 0.1 * rng.standard_normal(H)
    b3 = 0.05 * rng.standard_normal(3)
    # the library rounds weights to bf16 and keeps biases in FP32: hand the oracle the same values
    return [_bf16_array(W1), b1.astype(np.float32).astype(np.float64), _bf16_array(W2),
            b2.astype(np.float32).astype(np.float64), _bf16_array(W3), b3.astype(np.float32).astype(np.float64)]


SCALE = np.array([0.5, 1.25, 2.0], dtype=np.float32)


def _gpu_filter(sim, J, P):
    sim.J.copy_(torch.as_tensor(J, dtype=torch.float32))
    sim.set_denoiser(P, SCALE)
    sim.current_filter()
    torch.cuda.synchronize()
    return sim.J.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n", [(40, 12, 20), (16, 4, 8), (21, 7, 9)])
def test_denoiser_matches_oracle_periodic(n):
    rng = np.random.default_rng(11)
    J = (rng.standard_normal((3, n[2], n[1], n[0])) * SCALE[:, None, None, None]).astype(np.float32)
    P = _params(12)
    d = (0.2, 0.25, 0.3)
    sim = pic.Simulation(n, d, 0.05, jpost="denoiser")
    got = _gpu_filter(sim, J, P)
    ref, y = O.denoise(J.astype(np.float64), SCALE.astype(np.float64), P, d=d)
    assert np.abs(y).max() > 0.05                         # the network changes J
    assert rel_l2(got, ref) <= 1e-4
    g = O.make_grid(n, d, 0.05)
    B = O.binomial(g, J.astype(np.float64))
    assert rel_l2(got - B, ref - B) <= 3e-3              # the learned correction itself


def test_denoiser_matches_oracle_moving_window():
    n = (36, 8, 16)
    sim = pic.Simulation(n, (0.25, 0.5, 0.5), 0.25, solver="pd", bc_x=1, jpost="denoiser", max_particles=1)
    sim.add_empty_species(1)
    sim.set_window(0)
    P = _params(13)
    sim.set_denoiser(P, SCALE)
    sim.step(11)                                          # vacuum: fields stay zero, the origin moves
    shift, origin = sim.window_state()
    assert origin == 11 and shift == 11
    rng = np.random.default_rng(14)
    J = (rng.standard_normal((3, n[2], n[1], n[0])) * SCALE[:, None, None, None]).astype(np.float32)
    got = _gpu_filter(sim, J, P)
    ref, _ = O.denoise(J.astype(np.float64), SCALE.astype(np.float64), P, d=(0.25, 0.5, 0.5),
                       bc=("window", "periodic", "periodic"), origin=origin)
    assert rel_l2(got, ref) <= 1e-4


def test_denoiser_requires_weights_and_grid_mode():
    sim = pic.Simulation((16, 8, 8), (0.2, 0.2, 0.2), 0.05, jpost="denoiser")
    with pytest.raises(pic.PicError):
        sim.current_filter()                              # no weights yet
    plain = pic.Simulation((16, 8, 8), (0.2, 0.2, 0.2), 0.05)
    with pytest.raises(pic.PicError):
        plain.set_denoiser(_params(1), SCALE)             # grid made without the denoiser
    bad = _params(2)
    bad[0] = bad[0].copy()
    bad[0][0, 0, 0, 0, 0] = np.nan
    with pytest.raises(pic.PicError):
        sim.set_denoiser(bad, SCALE)


def test_denoised_step_equals_split_path():
    from paper_1204_0838_amd import inputs

    grid = inputs.Grid(n=(24, 12, 16), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    pl = inputs.uniform_random_plasma(grid, ppc=2, seed=21, temperature_ev=20000.0, ux_amp=0.1)
    P = _params(15)
    sims = []
    for _ in range(2):
        s = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", jpost="denoiser", max_particles=pl.count)
        s.add_particles(pl)
        s.set_denoiser(P, [0.05, 0.05, 0.05])
        sims.append(s)
    a, b = sims
    a.step(4)
    for _ in range(4):
        b.gather_push(0)
        b.deposit(0)
        b.field_step()
    for fa, fb in ((a.E, b.E), (a.B, b.B), (a.J, b.J)):
        assert torch.equal(fa, fb)
    assert float(a.E.abs().max()) > 0.0
