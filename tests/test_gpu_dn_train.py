"""Denoiser training on the matrix cores: loss and gradients against the
exact FP64 oracle (the GPU rounds inputs, activations and backward signals
to bf16, so agreement is to bf16 accuracy, not to round-off), and an Adam
run that learns a known linear filter."""
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


def _params(seed, amp=1.0):
    rng = np.random.default_rng(seed)
    W1 = amp * rng.standard_normal((32, 3, 3, 3, 3)) / np.sqrt(81.0)
    W2 = amp * rng.standard_normal((32, 32, 3, 3, 3)) / np.sqrt(864.0)
    W3 = amp * rng.standard_normal((3, 32, 3, 3, 3)) / np.sqrt(864.0)
    b1 = 0.1 * rng.standard_normal(32)
    b2 = 0.1 * rng.standard_normal(32)
    b3 = 0.05 * rng.standard_normal(3)
    return [_bf16_array(W1), b1.astype(np.float32).astype(np.float64), _bf16_array(W2),
            b2.astype(np.float32).astype(np.float64), _bf16_array(W3), b3.astype(np.float32).astype(np.float64)]


SCALE = np.array([0.5, 1.0, 2.0])


@pytest.mark.parametrize("crop", [(32, 8, 16), (20, 6, 10)])
def test_trainer_gradients_match_oracle(crop):
    nx, ny, nz = crop
    rng = np.random.default_rng(31)
    J = rng.standard_normal((3, nz, ny, nx)) * SCALE[:, None, None, None]
    T = J + 0.5 * rng.standard_normal((3, nz, ny, nx)) * SCALE[:, None, None, None]
    J = J.astype(np.float32)
    T = T.astype(np.float32)
    P = _params(32)
    d = (0.25, 0.5, 0.4)
    tr = pic.DenoiserTrainer(crop, cell=d)
    tr.set_params(P, SCALE)
    inp = torch.as_tensor(J).cuda().contiguous()
    tgt = torch.as_tensor(T).cuda().contiguous()
    loss, G = tr.grad(inp, tgt)
    s = SCALE[:, None, None, None]
    # the network's input is bf16(J / s) by definition; the rest of the
    # oracle's pass is exact (the GPU rounds activations and backward signals)
    x = _bf16_array(J.astype(np.float64) / s)
    ref_loss, ref_G = O.denoise_grad(J.astype(np.float64), x, T.astype(np.float64), SCALE, P, d=d,
                                     bc=("zero", "zero", "zero"))
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss
    for name, g, gr in zip(("W1", "b1", "W2", "b2", "W3", "b3"), G, ref_G):
        assert np.all(np.isfinite(g)), name
        assert rel_l2(g, gr) <= 3e-2, (name, rel_l2(g, gr))


def test_training_learns_a_divergence_free_correction():
    """Target: B(J) + sigma curl(J / s), which the network reaches with an
    identity path (relu(x) - relu(-x)); training from a small random start
    must cut the loss tenfold."""
    crop = (32, 8, 16)
    nx, ny, nz = crop
    d = (0.25, 0.5, 0.5)
    rng = np.random.default_rng(41)
    J = rng.standard_normal((3, nz, ny, nx))
    D = np.zeros((3, 3, 3))
    D[1, 1, 1] = 1.0
    Pid = [np.zeros((32, 3, 3, 3, 3)), np.zeros(32), np.zeros((32, 32, 3, 3, 3)), np.zeros(32),
           np.zeros((3, 32, 3, 3, 3)), np.zeros(3)]
    for c in range(3):
        Pid[0][c, c] = D
        Pid[0][3 + c, c] = -D
        Pid[2][c, c] = D
        Pid[2][3 + c, 3 + c] = D
        Pid[4][c, c] = D
        Pid[4][c, 3 + c] = -D
    T, _ = O.denoise(J, [1.0, 1.0, 1.0], Pid, d=d, bc=("zero", "zero", "zero"), round_bf16=False)
    tr = pic.DenoiserTrainer(crop, cell=d)
    tr.set_params(_params(42, amp=0.3), [1.0, 1.0, 1.0])
    inp = torch.as_tensor(J.astype(np.float32)).cuda().contiguous()
    tgt = torch.as_tensor(T.astype(np.float32)).cuda().contiguous()
    first = tr.step(inp, tgt, 2e-3)
    for _ in range(300):
        tr.step(inp, tgt, 2e-3, want_loss=False)
    last = tr.step(inp, tgt, 2e-3)
    assert np.isfinite(last) and last < 0.1 * first, (first, last)
    P = tr.get_params()
    assert all(np.all(np.isfinite(p)) for p in P)
    # the learned parameters plug into the production denoiser
    sim = pic.Simulation(crop, d, 0.1, jpost="denoiser")
    sim.set_denoiser(P, [1.0, 1.0, 1.0])


def test_batched_step_and_eval_agree_with_single_crop_losses():
    crop = (32, 8, 16)
    rng = np.random.default_rng(51)
    pairs = []
    for _ in range(3):
        J = rng.standard_normal((3, 16, 8, 32)).astype(np.float32)
        T = (J + 0.3 * rng.standard_normal(J.shape)).astype(np.float32)
        pairs.append((torch.as_tensor(J).cuda().contiguous(), torch.as_tensor(T).cuda().contiguous()))
    tr = pic.DenoiserTrainer(crop, cell=(0.25, 0.5, 0.5))
    tr.set_params(_params(52), SCALE)
    single = [tr.grad(a, b)[0] for a, b in pairs]
    ev = tr.eval([a for a, _ in pairs], [b for _, b in pairs])
    assert abs(ev - np.mean(single)) <= 1e-9 * max(1.0, ev)
    before = tr.step_batch([a for a, _ in pairs], [b for _, b in pairs], 1e-3)
    assert abs(before - ev) <= 1e-9 * max(1.0, ev)
    after = tr.eval([a for a, _ in pairs], [b for _, b in pairs])
    assert after < before                     # one Adam step on the mean gradient lowers the mean loss
    tr.freeze_biases(True)
    b0 = tr.get_params()[1].copy()
    tr.step_batch([a for a, _ in pairs], [b for _, b in pairs], 1e-3)
    assert np.array_equal(tr.get_params()[1], b0)


def test_trainer_gradients_on_a_crop_of_more_than_512_tiles():
    """A 100x42x60 crop has 7 x 11 x 8 = 616 output tiles of 16x4x8 cells, so
    the weight-gradient kernel (at most 512 workgroups) sums several tiles per
    workgroup: tile t and tile t + 512 in one.  The data sit in two boxes, one
    in tile 40 and one across tiles 551 and 552 (ragged tiles on the x and z
    faces), with zeros elsewhere; with zero biases nothing outside a box's
    7-cell neighbourhood is touched, so the crop's gradient is the sum of
    the gradients of two small crops around the boxes (each box plus an
    8-cell margin, cut at the crop's faces, where both see zero padding),
    weighted by their cell counts: the oracle computes those small crops."""
    crop = (100, 42, 60)
    nx, ny, nz = crop
    print(f"trainer gradients on a {crop} crop (616 tiles)", flush=True)
    rng = np.random.default_rng(61)
    J = np.zeros((3, nz, ny, nx))
    T = np.zeros_like(J)
    boxes = [((82, 90), (20, 24), (2, 6)), ((92, 100), (4, 8), (56, 60))]
    for (x0, x1), (y0, y1), (z0, z1) in boxes:
        shp = (3, z1 - z0, y1 - y0, x1 - x0)
        Jb = rng.standard_normal(shp) * SCALE[:, None, None, None]
        J[:, z0:z1, y0:y1, x0:x1] = Jb
        T[:, z0:z1, y0:y1, x0:x1] = Jb + 0.5 * rng.standard_normal(shp) * SCALE[:, None, None, None]
    J = J.astype(np.float32)
    T = T.astype(np.float32)
    P = _params(62)
    for k in (1, 3, 5):
        P[k] = np.zeros_like(P[k])
    d = (0.25, 0.5, 0.4)
    tr = pic.DenoiserTrainer(crop, cell=d)
    tr.set_params(P, SCALE)
    loss, G = tr.grad(torch.as_tensor(J).cuda().contiguous(), torch.as_tensor(T).cuda().contiguous())
    s = SCALE[:, None, None, None]
    n_big = nx * ny * nz
    ref_loss = 0.0
    ref_G = [np.zeros_like(p) for p in P]
    for (x0, x1), (y0, y1), (z0, z1) in boxes:
        sx = slice(max(0, x0 - 8), min(nx, x1 + 8))
        sy = slice(max(0, y0 - 8), min(ny, y1 + 8))
        sz = slice(max(0, z0 - 8), min(nz, z1 + 8))
        Js = np.ascontiguousarray(J[:, sz, sy, sx]).astype(np.float64)
        Ts = np.ascontiguousarray(T[:, sz, sy, sx]).astype(np.float64)
        n_small = Js.shape[1] * Js.shape[2] * Js.shape[3]
        ls, Gs = O.denoise_grad(Js, _bf16_array(Js / s), Ts, SCALE, P, d=d, bc=("zero", "zero", "zero"))
        ref_loss += ls * n_small / n_big
        for acc, g in zip(ref_G, Gs):
            acc += g * (n_small / n_big)
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss
    for name, g, gr in zip(("W1", "b1", "W2", "b2", "W3", "b3"), G, ref_G):
        assert np.all(np.isfinite(g)), name
        assert rel_l2(g, gr) <= 3e-2, (name, rel_l2(g, gr))
