"""Pins of the FP64 denoiser oracle against facts fixed by mathematics rather
than by the oracle itself: bfloat16 rounding of known values, the
convolution theorem (FFT) for periodic and zero-padded cross-correlation, a
shifted delta kernel, the separable binomial kernel against the (separately
pinned) binomial current filter, the moving-window seam, the binomial filter
as the zero-correction network, the vanishing divergence of the correction,
and finite differences of the training loss for every gradient."""
import numpy as np
import pytest

from oracle import oracle as O


def test_bf16_rounding_known_values():
    assert O.bf16(1.0) == 1.0
    assert O.bf16(1.0 + 2.0 ** -8) == 1.0                   # tie -> even (1.0000000)
    assert O.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6    # tie -> even (1.0000010)
    assert O.bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7        # representable
    assert O.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7   # above the tie
    assert O.bf16(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    assert O.bf16(3.14159) == 3.140625
    assert O.bf16(255.5) == 256.0 and O.bf16(254.5) == 254.0


def _fft_xcorr(inp, W, pad=None):
    """sum_a W[co, ci, a] in[ci](x + a) by the convolution theorem; optional zero padding per axis."""
    cin, nz, ny, nx = inp.shape
    if pad is not None:
        inp = np.pad(inp, [(0, 0)] + [(2, 2) if p else (0, 0) for p in pad[::-1]])
    shape = inp.shape[1:]
    F = np.fft.fftn(inp, axes=(1, 2, 3))
    out = []
    for co in range(W.shape[0]):
        acc = np.zeros(shape, complex)
        for ci in range(cin):
            K = np.zeros(shape)
            for c in range(3):
                for b in range(3):
                    for a in range(3):
                        K[(1 - c) % shape[0], (1 - b) % shape[1], (1 - a) % shape[2]] += W[co, ci, c, b, a]
            acc += F[ci] * np.fft.fftn(K)
        out.append(np.real(np.fft.ifftn(acc)))
    out = np.array(out)
    if pad is not None:
        sl = [slice(None)] + [slice(2, -2) if p else slice(None) for p in pad[::-1]]
        out = out[tuple(sl)]
    return out


def test_periodic_conv_matches_convolution_theorem():
    rng = np.random.default_rng(1)
    inp = rng.standard_normal((2, 4, 5, 6))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    got = O.conv3d(inp, W, b)
    ref = _fft_xcorr(inp, W) + b[:, None, None, None]
    assert np.abs(got - ref).max() < 1e-12


def test_zero_padded_conv_matches_convolution_theorem():
    rng = np.random.default_rng(2)
    inp = rng.standard_normal((2, 5, 4, 7))
    W = rng.standard_normal((2, 2, 3, 3, 3))
    got = O.conv3d(inp, W, None, bc=("zero", "periodic", "zero"))
    ref = _fft_xcorr(inp, W, pad=(True, False, True))
    assert np.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("dz,dy,dx", [(0, 0, 1), (1, 0, 0), (0, -1, 0), (1, 1, -1)])
def test_delta_kernel_shifts(dz, dy, dx):
    rng = np.random.default_rng(3)
    inp = rng.standard_normal((2, 4, 5, 6))
    W = np.zeros((2, 2, 3, 3, 3))
    for c in range(2):
        W[c, c, 1 + dz, 1 + dy, 1 + dx] = 1.0
    got = O.conv3d(inp, W)
    ref = np.roll(inp, shift=(-dz, -dy, -dx), axis=(1, 2, 3))     # out(x) = in(x + d)
    assert np.array_equal(got, ref)


def test_binomial_kernel_equals_binomial_filter():
    g = O.make_grid((7, 6, 5), (0.2, 0.2, 0.2), 0.05)
    rng = np.random.default_rng(4)
    J = rng.standard_normal((3, 5, 6, 7))
    w1 = np.array([0.25, 0.5, 0.25])
    k = np.einsum("i,j,k->ijk", w1, w1, w1)
    W = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        W[c, c] = k
    ref = O.binomial(g, J)
    assert np.abs(O.conv3d(J, W) - ref).max() < 1e-14


def test_window_seam_is_zero_padding_in_window_order():
    rng = np.random.default_rng(5)
    inp = rng.standard_normal((2, 3, 4, 9))
    W = rng.standard_normal((2, 2, 3, 3, 3))
    origin = 4
    got = O.conv3d(inp, W, bc=("window", "periodic", "periodic"), origin=origin)
    win = np.roll(inp, -origin, axis=3)            # window cell 0 first
    ref = np.roll(O.conv3d(win, W, bc=("zero", "periodic", "periodic")), origin, axis=3)
    assert np.abs(got - ref).max() < 1e-13


def _params(rng, H, amp=0.3):
    return [amp * rng.standard_normal((H, 3, 3, 3, 3)), 0.1 * rng.standard_normal(H),
            amp * rng.standard_normal((H, H, 3, 3, 3)), 0.1 * rng.standard_normal(H),
            amp * rng.standard_normal((3, H, 3, 3, 3)), 0.1 * rng.standard_normal(3)]


def test_zero_last_layer_is_the_binomial_filter():
    rng = np.random.default_rng(6)
    P = _params(rng, 4)
    P[4][:] = 0.0
    P[5][:] = 0.0
    J = rng.standard_normal((3, 3, 4, 5))
    g = O.make_grid((5, 4, 3), (0.2, 0.2, 0.2), 0.05)
    Jout, y = O.denoise(J, [2.0, 3.0, 0.5], P)
    assert np.abs(Jout - O.binomial(g, J)).max() < 1e-14 and not y.any()


@pytest.mark.parametrize("bc", [("periodic",) * 3])
def test_correction_is_divergence_free(bc):
    """The backward-difference divergence (the continuity equation's) of Jout - B(J) vanishes."""
    rng = np.random.default_rng(9)
    P = _params(rng, 4)
    d = (0.25, 0.5, 0.4)
    J = rng.standard_normal((3, 5, 6, 7))
    Jout, y = O.denoise(J, [1.0, 2.0, 0.5], P, d=d, bc=bc)
    P0 = [a.copy() for a in P]
    P0[4][:] = 0.0
    P0[5][:] = 0.0
    Jb, _ = O.denoise(J, [1.0, 2.0, 0.5], P0, d=d, bc=bc)
    C = Jout - Jb
    assert np.abs(C).max() > 0.1
    div = np.zeros(C.shape[1:])
    for a, axis in ((0, 2), (1, 1), (2, 0)):      # component a varies along array axis `axis` of [z, y, x]
        prev = np.roll(C[a], 1, axis=axis)
        if bc[a] == "zero":
            sl = [slice(None)] * 3
            sl[axis] = 0
            prev[tuple(sl)] = 0.0
        div += (C[a] - prev) / d[a]
    assert np.abs(div).max() < 1e-12 * np.abs(C).max() / min(d)


def test_correction_has_no_nyquist_content():
    """B removes the (pi, ., .) modes of the correction (checked on an even periodic grid)."""
    rng = np.random.default_rng(10)
    P = _params(rng, 4)
    J = rng.standard_normal((3, 4, 6, 8))
    Jout, _ = O.denoise(J, [1.0, 1.0, 1.0], P, d=(0.25, 0.5, 0.5))
    for axis in (1, 2, 3):
        sign = (-1.0) ** np.arange(J.shape[axis])
        shape = [1, 1, 1, 1]
        shape[axis] = -1
        assert np.abs((Jout * sign.reshape(shape)).sum(axis=axis)).max() < 1e-12


def test_denoise_rounds_input_and_scales_output():
    """With a single-tap identity network the output is the bf16 rounding of J/s, times s."""
    H = 3
    P = [np.zeros((H, 3, 3, 3, 3)), np.zeros(H), np.zeros((H, H, 3, 3, 3)), np.zeros(H),
         np.zeros((3, H, 3, 3, 3)), np.zeros(3)]
    for c in range(3):
        P[0][c, c, 1, 1, 1] = 1.0
        P[2][c, c, 1, 1, 1] = 1.0
        P[4][c, c, 1, 1, 1] = 1.0
    rng = np.random.default_rng(7)
    J = np.abs(rng.standard_normal((3, 2, 3, 4))) + 0.1     # positive: relu passes it
    s = np.array([0.7, 1.3, 2.1])
    _, y = O.denoise(J, s, P)
    ref = np.vectorize(O.bf16)(J / s[:, None, None, None])
    assert np.array_equal(y, ref)


def test_training_gradients_match_finite_differences():
    rng = np.random.default_rng(8)
    H = 3
    P = _params(rng, H)
    J = rng.standard_normal((3, 3, 3, 4))
    T = rng.standard_normal((3, 3, 3, 4))
    s = np.array([0.7, 1.0, 1.4])
    d = (0.25, 0.5, 0.4)
    bc = ("zero", "zero", "zero")
    x = J / s[:, None, None, None]
    loss, G = O.denoise_grad(J, x, T, s, P, d=d, bc=bc)

    def fwd(Q):
        Jout, _ = O.denoise(J, s, Q, d=d, bc=bc, round_bf16=False)
        return np.mean(((Jout - T) / s[:, None, None, None]) ** 2)

    assert abs(fwd(P) - loss) < 1e-13 * max(1.0, loss)
    h = 1e-6
    worst = 0.0
    for k, A in enumerate(P):
        flat = A.reshape(-1)
        idx = range(flat.size) if flat.size <= 30 else rng.choice(flat.size, 30, replace=False)
        for i in idx:
            keep = flat[i]
            flat[i] = keep + h
            lp = fwd(P)
            flat[i] = keep - h
            lm = fwd(P)
            flat[i] = keep
            fd = (lp - lm) / (2 * h)
            g = G[k].reshape(-1)[i]
            worst = max(worst, abs(fd - g) / max(1e-3, abs(g)))
    assert worst < 1e-5
