/*
 * FP64 reference of the learned current denoiser: a three-layer 3D
 * convolutional network applied to the deposited current J before the field
 * update, and the gradients of its training loss.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product path
 * never links, calls or includes anything from here, and this file includes
 * nothing from the product path.
 *
 * The denoiser is not part of the paper.  The paper's own remedy for
 * particle noise in the current is the third-order (cubic) particle shape
 * (Sections 1 and 3.1); its runs use many particles per cell.  This network
 * is the library's learned stand-in for the plain binomial current filter at
 * a low particle count, defined here in full:
 *
 *   x    = bf16(J_d / s_d)                      (3 channels, s_d a fixed scale)
 *   a1   = bf16(relu(conv(x,  W1) + b1))        (H channels)
 *   a2   = bf16(relu(conv(a1, W2) + b2))        (H channels)
 *   y    = conv(a2, W3) + b3                    (3 channels)
 *   Jout = J_d + s_d y_d                        (a residual correction)
 *
 * conv is the 3x3x3 cross-correlation with "same" output size:
 *   out[co](i,j,k) = sum_ci sum_{a,b,c in -1..1} W[co][ci][c+1][b+1][a+1] in[ci](i+a, j+b, k+c)
 * (weights indexed [out][in][z][y][x]).  Neighbours outside the grid follow a
 * per-axis rule: periodic, zero outside [0, n), or -- x only, moving window --
 * zero across the seam where the window's two ends meet in the circular
 * buffer (window cell xw = (i - origin) mod n, neighbours with xw + a outside
 * [0, n) are zero).  bf16() rounds to the nearest bfloat16 (8 significant
 * bits), ties to even; with `round` = 0 it is the identity (the training
 * loss and its gradients are exact FP64).
 *
 * Training loss: mean over cells and the 3 output channels of (y - r)^2
 * with r the target residual (J_target - J) / s, i.e. the squared error of
 * Jout against J_target in units of s.  Gradients by reverse-mode
 * differentiation of the definition above, layer by layer: the adjoint of
 * a conv scatters each output's gradient back to the inputs it read.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_BC_PERIODIC = 0, ORA_BC_ZERO = 1, ORA_BC_WINDOW = 2 };

/* Round to the nearest bfloat16 value, ties to even (normal range). */
double ora_bf16(double x) {
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    const double m = frexp(x, &e);          /* x = m 2^e, 0.5 <= |m| < 1 */
    const double q = nearbyint(m * 256.0);  /* 8 significant bits; default rounding is to nearest even */
    return ldexp(q / 256.0, e);
}

/* Linear index of the neighbour (i+a, j+b, k+c) of cell (i,j,k), or -1 when
 * the neighbour reads as zero. */
static int64_t neighbour(const int64_t n[3], const int32_t bc[3], int64_t origin, int64_t i, int64_t j, int64_t k,
                         int a, int b, int c) {
    int64_t p[3] = {i + a, j + b, k + c};
    const int64_t q[3] = {i, j, k};
    const int off[3] = {a, b, c};
    for (int d = 0; d < 3; ++d) {
        if (bc[d] == ORA_BC_PERIODIC) {
            p[d] = ((p[d] % n[d]) + n[d]) % n[d];
        } else if (bc[d] == ORA_BC_ZERO) {
            if (p[d] < 0 || p[d] >= n[d]) return -1;
        } else {   /* moving-window seam (x) */
            const int64_t xw = ((q[d] - origin) % n[d] + n[d]) % n[d];
            const int64_t t = xw + off[d];
            if (t < 0 || t >= n[d]) return -1;
            p[d] = (t + origin) % n[d];
        }
    }
    return p[0] + n[0] * (p[1] + n[1] * p[2]);
}

static double wat(const double *W, int cin, int co, int ci, int a, int b, int c) {
    return W[(((int64_t)co * cin + ci) * 3 + (c + 1)) * 9 + (b + 1) * 3 + (a + 1)];
}

/* out[co][cell] = bias[co] + sum over inputs and taps (definition above). */
void ora_conv3d(const int64_t n[3], const int32_t bc[3], int64_t origin, const double *in, int cin,
                const double *W, const double *bias, int cout, double *out) {
    const int64_t N = n[0] * n[1] * n[2];
    for (int co = 0; co < cout; ++co)
        for (int64_t k = 0; k < n[2]; ++k)
            for (int64_t j = 0; j < n[1]; ++j)
                for (int64_t i = 0; i < n[0]; ++i) {
                    double s = bias ? bias[co] : 0.0;
                    for (int ci = 0; ci < cin; ++ci)
                        for (int c = -1; c <= 1; ++c)
                            for (int b = -1; b <= 1; ++b)
                                for (int a = -1; a <= 1; ++a) {
                                    const int64_t p = neighbour(n, bc, origin, i, j, k, a, b, c);
                                    if (p >= 0) s += wat(W, cin, co, ci, a, b, c) * in[(int64_t)ci * N + p];
                                }
                    out[(int64_t)co * N + i + n[0] * (j + n[1] * k)] = s;
                }
}

/* Adjoint of ora_conv3d with respect to its input: din += conv^T(dout). */
static void conv_back_data(const int64_t n[3], const int32_t bc[3], int64_t origin, double *din, int cin,
                           const double *W, int cout, const double *dout) {
    const int64_t N = n[0] * n[1] * n[2];
    for (int co = 0; co < cout; ++co)
        for (int64_t k = 0; k < n[2]; ++k)
            for (int64_t j = 0; j < n[1]; ++j)
                for (int64_t i = 0; i < n[0]; ++i) {
                    const double g = dout[(int64_t)co * N + i + n[0] * (j + n[1] * k)];
                    for (int ci = 0; ci < cin; ++ci)
                        for (int c = -1; c <= 1; ++c)
                            for (int b = -1; b <= 1; ++b)
                                for (int a = -1; a <= 1; ++a) {
                                    const int64_t p = neighbour(n, bc, origin, i, j, k, a, b, c);
                                    if (p >= 0) din[(int64_t)ci * N + p] += wat(W, cin, co, ci, a, b, c) * g;
                                }
                }
}

/* Gradient with respect to the weights and biases: dW += dout x in (per tap), db += dout. */
static void conv_back_weights(const int64_t n[3], const int32_t bc[3], int64_t origin, const double *in, int cin,
                              int cout, const double *dout, double *dW, double *db) {
    const int64_t N = n[0] * n[1] * n[2];
    for (int co = 0; co < cout; ++co)
        for (int64_t k = 0; k < n[2]; ++k)
            for (int64_t j = 0; j < n[1]; ++j)
                for (int64_t i = 0; i < n[0]; ++i) {
                    const double g = dout[(int64_t)co * N + i + n[0] * (j + n[1] * k)];
                    db[co] += g;
                    for (int ci = 0; ci < cin; ++ci)
                        for (int c = -1; c <= 1; ++c)
                            for (int b = -1; b <= 1; ++b)
                                for (int a = -1; a <= 1; ++a) {
                                    const int64_t p = neighbour(n, bc, origin, i, j, k, a, b, c);
                                    if (p >= 0)
                                        dW[(((int64_t)co * cin + ci) * 3 + (c + 1)) * 9 + (b + 1) * 3 + (a + 1)] +=
                                            g * in[(int64_t)ci * N + p];
                                }
                }
}

static double *dalloc(int64_t count) { return (double *)calloc((size_t)(count > 0 ? count : 1), sizeof(double)); }

static void relu_round(double *a, int64_t count, int round) {
    for (int64_t q = 0; q < count; ++q) {
        const double v = a[q] > 0.0 ? a[q] : 0.0;
        a[q] = round ? ora_bf16(v) : v;
    }
}

/* Forward pass.  J: [3][N] current; scale[3]; hidden H; weights as above.
 * Outputs: Jout [3][N] (may be NULL), y [3][N] (may be NULL).  round != 0
 * applies the bf16 roundings of the definition (weights are used as given).
 * Returns 0, or -1 when memory runs out. */
int ora_denoise(const int64_t n[3], const int32_t bc[3], int64_t origin, const double *J, const double scale[3],
                int hidden, const double *W1, const double *b1, const double *W2, const double *b2,
                const double *W3, const double *b3, int round, double *Jout, double *y_out) {
    const int64_t N = n[0] * n[1] * n[2];
    double *x = dalloc(3 * N), *a1 = dalloc(hidden * N), *a2 = dalloc(hidden * N), *y = dalloc(3 * N);
    if (!x || !a1 || !a2 || !y) {
        free(x), free(a1), free(a2), free(y);
        return -1;
    }
    for (int d = 0; d < 3; ++d)
        for (int64_t q = 0; q < N; ++q) {
            const double v = J[d * N + q] / scale[d];
            x[d * N + q] = round ? ora_bf16(v) : v;
        }
    ora_conv3d(n, bc, origin, x, 3, W1, b1, hidden, a1);
    relu_round(a1, hidden * N, round);
    ora_conv3d(n, bc, origin, a1, hidden, W2, b2, hidden, a2);
    relu_round(a2, hidden * N, round);
    ora_conv3d(n, bc, origin, a2, hidden, W3, b3, 3, y);
    for (int d = 0; d < 3; ++d)
        for (int64_t q = 0; q < N; ++q) {
            if (Jout) Jout[d * N + q] = J[d * N + q] + scale[d] * y[d * N + q];
            if (y_out) y_out[d * N + q] = y[d * N + q];
        }
    free(x), free(a1), free(a2), free(y);
    return 0;
}

/* Training loss and its exact gradients (no rounding).  x: [3][N] scaled
 * input, r: [3][N] target residual.  Gradient outputs have the shapes of
 * the weights and biases and are overwritten.  Returns the loss (NaN when
 * memory runs out). */
double ora_denoise_grad(const int64_t n[3], const int32_t bc[3], int64_t origin, const double *x, const double *r,
                        int hidden, const double *W1, const double *b1, const double *W2, const double *b2,
                        const double *W3, const double *b3, double *gW1, double *gb1, double *gW2, double *gb2,
                        double *gW3, double *gb3) {
    const int64_t N = n[0] * n[1] * n[2];
    const int H = hidden;
    double *z1 = dalloc(H * N), *a1 = dalloc(H * N), *z2 = dalloc(H * N), *a2 = dalloc(H * N);
    double *y = dalloc(3 * N), *dy = dalloc(3 * N), *da2 = dalloc(H * N), *da1 = dalloc(H * N);
    if (!z1 || !a1 || !z2 || !a2 || !y || !dy || !da2 || !da1) {
        free(z1), free(a1), free(z2), free(a2), free(y), free(dy), free(da2), free(da1);
        return NAN;
    }
    ora_conv3d(n, bc, origin, x, 3, W1, b1, H, z1);
    for (int64_t q = 0; q < H * N; ++q) a1[q] = z1[q] > 0.0 ? z1[q] : 0.0;
    ora_conv3d(n, bc, origin, a1, H, W2, b2, H, z2);
    for (int64_t q = 0; q < H * N; ++q) a2[q] = z2[q] > 0.0 ? z2[q] : 0.0;
    ora_conv3d(n, bc, origin, a2, H, W3, b3, 3, y);
    double loss = 0.0;
    const double inv = 1.0 / (3.0 * (double)N);
    for (int64_t q = 0; q < 3 * N; ++q) {
        const double e = y[q] - r[q];
        loss += e * e * inv;
        dy[q] = 2.0 * e * inv;
    }
    memset(gW1, 0, sizeof(double) * (size_t)H * 3 * 27);
    memset(gW2, 0, sizeof(double) * (size_t)H * H * 27);
    memset(gW3, 0, sizeof(double) * (size_t)3 * H * 27);
    memset(gb1, 0, sizeof(double) * (size_t)H);
    memset(gb2, 0, sizeof(double) * (size_t)H);
    memset(gb3, 0, sizeof(double) * 3);
    /* layer 3 */
    conv_back_weights(n, bc, origin, a2, H, 3, dy, gW3, gb3);
    conv_back_data(n, bc, origin, da2, H, W3, 3, dy);
    for (int64_t q = 0; q < H * N; ++q) da2[q] = z2[q] > 0.0 ? da2[q] : 0.0;   /* through relu: dz2 */
    /* layer 2 */
    conv_back_weights(n, bc, origin, a1, H, H, da2, gW2, gb2);
    conv_back_data(n, bc, origin, da1, H, W2, H, da2);
    for (int64_t q = 0; q < H * N; ++q) da1[q] = z1[q] > 0.0 ? da1[q] : 0.0;   /* dz1 */
    /* layer 1 */
    conv_back_weights(n, bc, origin, x, 3, H, da1, gW1, gb1);
    free(z1), free(a1), free(z2), free(a2), free(y), free(dy), free(da2), free(da1);
    return loss;
}
