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
 *   Jout = B(J + sigma curl(y))                 (binomial filter of the current
 *                                               plus a divergence-free correction)
 *
 * B is one (1/4, 1/2, 1/4) pass along each axis (the 27-point product
 * stencil) on each component.  curl is the discrete curl with backward
 * differences, the one the E update applies to B (Section 1):
 *   curl(y)_x = (y_z - y_z[j-1]) / dy - (y_y - y_y[k-1]) / dz, and cyclic;
 * the backward-difference divergence that the continuity equation uses
 * annihilates it exactly, and on a periodic grid B commutes with it, so
 * Jout satisfies the same discrete continuity equation as B(J).  Filtering
 * the correction as well keeps it free of the grid-scale (Nyquist) modes
 * that B removes from J.  sigma = dx (s_x + s_y + s_z) / 3.  With y = 0 the
 * network is the binomial filter.
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
 * Training loss: mean over cells and the 3 components of
 * ((Jout_d - J_target_d) / s_d)^2.  Gradients by reverse-mode
 * differentiation of the definition above, layer by layer: the adjoint of
 * a conv (or of the curl) scatters each output's gradient back to the
 * inputs it read.
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

/* Binomial filter of each of the 3 components (same boundary rule). */
static void binomial3(const int64_t n[3], const int32_t bc[3], int64_t origin, const double *J, double *out) {
    const int64_t N = n[0] * n[1] * n[2];
    const double w[3] = {0.25, 0.5, 0.25};
    for (int d = 0; d < 3; ++d)
        for (int64_t k = 0; k < n[2]; ++k)
            for (int64_t j = 0; j < n[1]; ++j)
                for (int64_t i = 0; i < n[0]; ++i) {
                    double acc = 0.0;
                    for (int c = -1; c <= 1; ++c)
                        for (int b = -1; b <= 1; ++b)
                            for (int a = -1; a <= 1; ++a) {
                                const int64_t p = neighbour(n, bc, origin, i, j, k, a, b, c);
                                if (p >= 0) acc += w[a + 1] * w[b + 1] * w[c + 1] * J[d * N + p];
                            }
                    out[d * N + i + n[0] * (j + n[1] * k)] = acc;
                }
}

/* The backward-difference curl's terms: component `out` at cell c gets
 * +y_t2(c)/d_t1 - y_t2(c - e_t1)/d_t1 - y_t1(c)/d_t2 + y_t1(c - e_t2)/d_t2
 * with (t1, t2) = the other two axes in cyclic order.  `adjoint` = 0 adds
 * sigma curl(y) to J; 1 scatters sigma curl^T(g) into y (y += ...). */
static void curl_terms(const int64_t n[3], const int32_t bc[3], int64_t origin, const double d[3], double sigma,
                       double *y, double *J, const double *g, int adjoint) {
    const int64_t N = n[0] * n[1] * n[2];
    for (int comp = 0; comp < 3; ++comp) {
        const int t1 = (comp + 1) % 3, t2 = (comp + 2) % 3;
        for (int64_t k = 0; k < n[2]; ++k)
            for (int64_t j = 0; j < n[1]; ++j)
                for (int64_t i = 0; i < n[0]; ++i) {
                    const int64_t c = i + n[0] * (j + n[1] * k);
                    int o1[3] = {0, 0, 0}, o2[3] = {0, 0, 0};
                    o1[t1] = -1;
                    o2[t2] = -1;
                    const int64_t m1 = neighbour(n, bc, origin, i, j, k, o1[0], o1[1], o1[2]);
                    const int64_t m2 = neighbour(n, bc, origin, i, j, k, o2[0], o2[1], o2[2]);
                    /* four terms: (source component, source cell, coefficient) */
                    const int sc[4] = {t2, t2, t1, t1};
                    const int64_t cell[4] = {c, m1, c, m2};
                    const double coef[4] = {sigma / d[t1], -sigma / d[t1], -sigma / d[t2], sigma / d[t2]};
                    for (int q = 0; q < 4; ++q) {
                        if (cell[q] < 0) continue;
                        if (!adjoint)
                            J[comp * N + c] += coef[q] * y[sc[q] * N + cell[q]];
                        else
                            y[sc[q] * N + cell[q]] += coef[q] * g[comp * N + c];
                    }
                }
    }
}

double ora_denoise_sigma(const double d[3], const double scale[3]) {
    return d[0] * (scale[0] + scale[1] + scale[2]) / 3.0;
}

/* Forward pass.  J: [3][N] current; d: cell sizes; scale[3]; hidden H;
 * weights as above.  Outputs: Jout [3][N] (may be NULL), y [3][N] (may be
 * NULL).  round != 0 applies the bf16 roundings of the definition (weights
 * are used as given).  Returns 0, or -1 when memory runs out. */
int ora_denoise(const int64_t n[3], const int32_t bc[3], int64_t origin, const double d[3], const double *J,
                const double scale[3], int hidden, const double *W1, const double *b1, const double *W2,
                const double *b2, const double *W3, const double *b3, int round, double *Jout, double *y_out) {
    const int64_t N = n[0] * n[1] * n[2];
    double *x = dalloc(3 * N), *a1 = dalloc(hidden * N), *a2 = dalloc(hidden * N), *y = dalloc(3 * N);
    double *o = dalloc(3 * N);
    if (!x || !a1 || !a2 || !y || !o) {
        free(x), free(a1), free(a2), free(y), free(o);
        return -1;
    }
    for (int c = 0; c < 3; ++c)
        for (int64_t q = 0; q < N; ++q) {
            const double v = J[c * N + q] / scale[c];
            x[c * N + q] = round ? ora_bf16(v) : v;
        }
    ora_conv3d(n, bc, origin, x, 3, W1, b1, hidden, a1);
    relu_round(a1, hidden * N, round);
    ora_conv3d(n, bc, origin, a1, hidden, W2, b2, hidden, a2);
    relu_round(a2, hidden * N, round);
    ora_conv3d(n, bc, origin, a2, hidden, W3, b3, 3, y);
    memcpy(x, J, sizeof(double) * 3 * (size_t)N);           /* x now holds J + sigma curl(y) */
    curl_terms(n, bc, origin, d, ora_denoise_sigma(d, scale), y, x, NULL, 0);
    binomial3(n, bc, origin, x, o);
    for (int64_t q = 0; q < 3 * N; ++q) {
        if (Jout) Jout[q] = o[q];
        if (y_out) y_out[q] = y[q];
    }
    free(x), free(a1), free(a2), free(y), free(o);
    return 0;
}

/* Training loss and its exact gradients.  J: [3][N] input current, x: [3][N]
 * the network's input (bf16(J/s) by the definition; passed in so that the
 * rounding is the caller's), T: [3][N] target current.  Gradient outputs
 * have the shapes of the weights and biases and are overwritten.  Returns
 * the loss (NaN when memory runs out). */
double ora_denoise_grad(const int64_t n[3], const int32_t bc[3], int64_t origin, const double d[3], const double *J,
                        const double *x, const double *T, const double scale[3], int hidden, const double *W1,
                        const double *b1, const double *W2, const double *b2, const double *W3, const double *b3,
                        double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3) {
    const int64_t N = n[0] * n[1] * n[2];
    const int H = hidden;
    double *z1 = dalloc(H * N), *a1 = dalloc(H * N), *z2 = dalloc(H * N), *a2 = dalloc(H * N);
    double *y = dalloc(3 * N), *dy = dalloc(3 * N), *da2 = dalloc(H * N), *da1 = dalloc(H * N);
    double *o = dalloc(3 * N), *go = dalloc(3 * N);
    if (!z1 || !a1 || !z2 || !a2 || !y || !dy || !da2 || !da1 || !o || !go) {
        free(z1), free(a1), free(z2), free(a2), free(y), free(dy), free(da2), free(da1), free(o), free(go);
        return NAN;
    }
    const double sigma = ora_denoise_sigma(d, scale);
    ora_conv3d(n, bc, origin, x, 3, W1, b1, H, z1);
    for (int64_t q = 0; q < H * N; ++q) a1[q] = z1[q] > 0.0 ? z1[q] : 0.0;
    ora_conv3d(n, bc, origin, a1, H, W2, b2, H, z2);
    for (int64_t q = 0; q < H * N; ++q) a2[q] = z2[q] > 0.0 ? z2[q] : 0.0;
    ora_conv3d(n, bc, origin, a2, H, W3, b3, 3, y);
    double *t = dalloc(3 * N);
    if (!t) {
        free(z1), free(a1), free(z2), free(a2), free(y), free(dy), free(da2), free(da1), free(o), free(go);
        return NAN;
    }
    memcpy(t, J, sizeof(double) * 3 * (size_t)N);
    curl_terms(n, bc, origin, d, sigma, y, t, NULL, 0);
    binomial3(n, bc, origin, t, o);
    double loss = 0.0;
    const double inv = 1.0 / (3.0 * (double)N);
    for (int c = 0; c < 3; ++c)
        for (int64_t q = 0; q < N; ++q) {
            const double e = (o[c * N + q] - T[c * N + q]) / scale[c];
            loss += e * e * inv;
            go[c * N + q] = 2.0 * e * inv / scale[c];
        }
    binomial3(n, bc, origin, go, t);                        /* B is symmetric: B^T go = B go */
    curl_terms(n, bc, origin, d, sigma, dy, NULL, t, 1);    /* dy = sigma curl^T(B go) */
    free(t);
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
    free(z1), free(a1), free(z2), free(a2), free(y), free(dy), free(da2), free(da1), free(o), free(go);
    return loss;
}
