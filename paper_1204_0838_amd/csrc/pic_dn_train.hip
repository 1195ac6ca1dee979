// Training of the learned current denoiser on the matrix cores.
//
// One training step on a crop of the current (zero beyond the crop's faces):
//   forward   a1 = bf16(relu(conv(x, W1) + b1)), a2 = ..., y = conv(a2, W3) + b3,
//             J' = B(J + sigma curl(y))
//   loss      mean over cells and 3 components of ((J' - J_target) / s)^2
//   backward  g = dL/dJ' = 2 (J' - J_target) / (3 N s^2), dy = sigma curl^T(B g)
//             dW3 = sum_cells dy x a2(shifted),   dz2 = conv^T(dy, W3) . [a2 > 0]
//             dW2 = sum_cells dz2 x a1(shifted),  dz1 = conv^T(dz2, W2) . [a1 > 0]
//             dW1 = sum_cells dz1 x x(shifted)
//   update    Adam on FP32 master weights, then bf16 repacking.
// conv^T is a convolution with mirrored taps (tap t -> 26 - t) and swapped
// channel roles, so the backward passes reuse the forward layer kernels.
// Weight gradients are GEMMs with the cells as the reduction dimension:
// dW[co][n] = sum_cells dout[cell][co] in[cell + offset(tap n)][channel n],
// n = tap * CIN + channel; each workgroup reduces tiles of 512 cells on the
// MFMA units and adds its partial sums to the FP32 gradient with atomics.
#include <math.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_dn_common.h"

namespace pic {

struct WgArgs {
    int n[3];
    int bc[3];
    const __bf16* in;     // [cell][CIN] bf16 (unless the input is the scaled current)
    const float* J[3];    // scaled-current input (layer 1)
    float inv_scale[3];
    const __bf16* dout;   // [cell][DC] bf16
    float* dW;            // [16 MB][NPAD] FP32
    float* db;            // [DC] FP32
    int ntiles;
};

// Flat tile index -> tile origin.
__device__ __forceinline__ void wg_tile(const WgArgs& a, int t, int t0[3]) {
    const int gx = (a.n[0] + DN_TX - 1) / DN_TX, gy = (a.n[1] + DN_TY - 1) / DN_TY;
    t0[0] = (t % gx) * DN_TX;
    t0[1] = ((t / gx) % gy) * DN_TY;
    t0[2] = (t / (gx * gy)) * DN_TZ;
}

__device__ __forceinline__ int wg_src(const WgArgs& a, const int t0[3], int hx, int hy, int hz) {
    const int x = dn_axis(t0[0] - 1 + hx, a.n[0], a.bc[0], 0);
    const int y = dn_axis(t0[1] - 1 + hy, a.n[1], a.bc[1], 0);
    const int z = dn_axis(t0[2] - 1 + hz, a.n[2], a.bc[2], 0);
    if (x < 0 || y < 0 || z < 0) return -1;
    return x + a.n[0] * (y + a.n[1] * z);
}

template <int CIN, int DC, int MB, bool INJ>
__global__ void __launch_bounds__(DN_THREADS) k_dn_wgrad(WgArgs a) {
    constexpr int NB = (27 * CIN + 15) / 16;          // 16-column blocks of n
    constexpr int NPAIR = MB * NB;
    constexpr int PW = (NPAIR + 7) / 8;               // (mb, nb) pairs per wavefront
    extern __shared__ __attribute__((aligned(16))) char wlds[];
    __bf16* in_l = reinterpret_cast<__bf16*>(wlds);                         // [halo cell][CIN]
    __bf16* do_l = reinterpret_cast<__bf16*>(wlds + DN_HCELLS * CIN * 2);  // [tile cell][DC]
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = l & 15, q = l >> 4;
    // per pair: halo offset of the tap, channel, validity
    int pdel[PW], pci[PW], pmb[PW];
    bool pok[PW];
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const int p = w + 8 * i;
        const int mb = p / NB, nb = p % NB;
        const int nn = nb * 16 + m;
        const int tap = nn / CIN;
        pok[i] = p < NPAIR && tap < 27;
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        pdel[i] = (dz * DN_HY + dy) * DN_HX + dx;
        pci[i] = nn % CIN;
        pmb[i] = mb;
    }
    f32x4 acc[PW];
#pragma unroll
    for (int i = 0; i < PW; ++i) acc[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        int t0[3];
        wg_tile(a, t, t0);
        __syncthreads();   // the previous tile's reads are done
        for (int c = threadIdx.x; c < DN_HCELLS; c += DN_THREADS) {
            const int hx = c % DN_HX, r = c / DN_HX, hy = r % DN_HY, hz = r / DN_HY;
            const int s = hx < DN_TX + 2 ? wg_src(a, t0, hx, hy, hz) : -1;
            if (INJ) {
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    in_l[c * CIN + d] = (__bf16)(s >= 0 && d < 3 ? a.J[d][s] * a.inv_scale[d] : 0.0f);
            } else {
                const uint4* src = reinterpret_cast<const uint4*>(a.in + (size_t)(s >= 0 ? s : 0) * CIN);
                uint4* dst = reinterpret_cast<uint4*>(in_l + c * CIN);
#pragma unroll
                for (int k = 0; k < CIN / 8; ++k) dst[k] = s >= 0 ? src[k] : make_uint4(0u, 0u, 0u, 0u);
            }
        }
        for (int c = threadIdx.x; c < DN_TX * DN_TY * DN_TZ; c += DN_THREADS) {
            const int lx = c % DN_TX, r = c / DN_TX, ly = r % DN_TY, lz = r / DN_TY;
            const int x = t0[0] + lx, y = t0[1] + ly, z = t0[2] + lz;
            const bool inside = x < a.n[0] && y < a.n[1] && z < a.n[2];
            const size_t s = inside ? (size_t)x + a.n[0] * ((size_t)y + (size_t)a.n[1] * z) : 0;
            if (DC == 4) {
                const uint2 v = inside ? reinterpret_cast<const uint2*>(a.dout)[s] : make_uint2(0u, 0u);
                reinterpret_cast<uint2*>(do_l)[c] = v;
            } else {
                const uint4* src = reinterpret_cast<const uint4*>(a.dout + s * DC);
                uint4* dst = reinterpret_cast<uint4*>(do_l + c * DC);
#pragma unroll
                for (int k = 0; k < DC / 8; ++k) dst[k] = inside ? src[k] : make_uint4(0u, 0u, 0u, 0u);
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < DC)
            for (int c = 0; c < DN_TX * DN_TY * DN_TZ; ++c) bsum += (float)do_l[c * DC + threadIdx.x];
        for (int ch = 0; ch < DN_TX * DN_TY * DN_TZ / 32; ++ch) {
            // K elements of this lane: tile cells 32 ch + 8 q + j, j = 0..7 (one x-row half)
            const int row = 2 * ch + (q >> 1);
            const int lz = row / DN_TY, ly = row % DN_TY, lx0 = 8 * (q & 1);
            const int hbase = (lz * DN_HY + ly) * DN_HX + lx0;
            const int cbase = row * DN_TX + lx0;
            bf16x8 A[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int co = mb * 16 + m;
#pragma unroll
                for (int j = 0; j < 8; ++j) A[mb][j] = co < DC ? do_l[(cbase + j) * DC + co] : (__bf16)0.0f;
            }
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                if (w + 8 * i >= NPAIR) break;
                bf16x8 B;
#pragma unroll
                for (int j = 0; j < 8; ++j) B[j] = pok[i] ? in_l[(hbase + j + pdel[i]) * CIN + pci[i]] : (__bf16)0.0f;
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[pmb[i]], B, acc[i], 0, 0, 0);
            }
        }
    }
    constexpr int NPAD = NB * 16;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const int p = w + 8 * i;
        if (p >= NPAIR) break;
        const int nn = (p % NB) * 16 + m;
        if (nn >= 27 * CIN) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = pmb[i] * 16 + 4 * q + j;
            if (co < DC) atomicAdd(a.dW + (size_t)co * NPAD + nn, acc[i][j]);
        }
    }
    if ((int)threadIdx.x < DC) atomicAdd(a.db + threadIdx.x, bsum);
}

// ---- parameters -------------------------------------------------------------
// Canonical FP32 parameter vector (the pic_denoiser_set layout):
//   W1 [32][3][27], W2 [32][32][27], W3 [3][32][27], b1 [32], b2 [32], b3 [3]
constexpr int kP_W1 = 0, kP_W2 = kP_W1 + 32 * 3 * 27, kP_W3 = kP_W2 + 32 * 32 * 27, kP_B1 = kP_W3 + 3 * 32 * 27,
              kP_B2 = kP_B1 + 32, kP_B3 = kP_B2 + 32, kP_N = kP_B3 + 3;
// Gradient buffers (FP32): dW1 [32][112], dW2 [32][864], dW3 [16][864] (rows < 4 used), db1 [32], db2 [32], db3 [4]
constexpr int kG_W1 = 0, kG_W2 = kG_W1 + 32 * 112, kG_W3 = kG_W2 + 32 * 864, kG_B1 = kG_W3 + 16 * 864,
              kG_B2 = kG_B1 + 32, kG_B3 = kG_B2 + 32, kG_N = kG_B3 + 4;
// bf16 packs: forward W1p [32][128], W2p [27][32][32], W3p [9 zx][6 r][16 (blk, co)][32] (the folded
// last layer: column 4 blk + co of fragment (zx, r) carries tap (dz, r - blk, dx));
// backward W3T [32][128] (k = tap * 4 + c: W3[c][co][26 - tap]), W2T [27][32][32] (W2[ci][co][26 - t])
constexpr int kK_W1 = 0, kK_W2 = kK_W1 + 32 * 128, kK_W3 = kK_W2 + 27 * 32 * 32, kK_W3T = kK_W3 + 9 * 6 * 16 * 32,
              kK_W2T = kK_W3T + 32 * 128, kK_N = kK_W2T + 27 * 32 * 32;
// FP32 biases of the kernels: b1 [32], b2 [32], b3 [16]
constexpr int kB_N = 80;

__device__ __forceinline__ int grad_index(int i) {
    if (i < kP_W2) {
        const int co = i / 81, r = i % 81, ci = r / 27, t = r % 27;
        return kG_W1 + co * 112 + t * 4 + ci;
    }
    if (i < kP_W3) {
        const int j = i - kP_W2, co = j / 864, r = j % 864, ci = r / 27, t = r % 27;
        return kG_W2 + co * 864 + t * 32 + ci;
    }
    if (i < kP_B1) {
        const int j = i - kP_W3, co = j / 864, r = j % 864, ci = r / 27, t = r % 27;
        return kG_W3 + co * 864 + t * 32 + ci;
    }
    if (i < kP_B2) return kG_B1 + (i - kP_B1);
    if (i < kP_B3) return kG_B2 + (i - kP_B2);
    return kG_B3 + (i - kP_B3);
}

// Adam step (when lr > 0) on the master weights, then write the bf16 packs
// and FP32 kernel biases of every parameter.
__global__ void k_dn_adam_pack(float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
                               const float* __restrict__ G, __bf16* __restrict__ K, float* __restrict__ Bk, float lr,
                               float c1, float c2, float gscale, int train_bias) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kP_N) return;
    float p = P[i];
    if (lr > 0.0f && (train_bias || i < kP_B1)) {
        const float g = G[grad_index(i)] * gscale;
        const float m = 0.9f * M[i] + 0.1f * g;
        const float v = 0.999f * V[i] + 0.001f * g * g;
        M[i] = m;
        V[i] = v;
        p -= lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
        P[i] = p;
    }
    const __bf16 b = (__bf16)p;
    if (i < kP_W2) {
        const int co = i / 81, r = i % 81, ci = r / 27, t = r % 27;
        K[kK_W1 + co * 128 + t * 4 + ci] = b;
    } else if (i < kP_W3) {
        const int j = i - kP_W2, co = j / 864, r = j % 864, ci = r / 27, t = r % 27;
        K[kK_W2 + (t * 32 + co) * 32 + ci] = b;
        K[kK_W2T + ((26 - t) * 32 + ci) * 32 + co] = b;
    } else if (i < kP_B1) {
        const int j = i - kP_W3, co = j / 864, r = j % 864, ci = r / 27, t = r % 27;
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
            K[kK_W3 + (((dz * 3 + dx) * 6 + blk + dy) * 16 + blk * 4 + co) * 32 + ci] = b;
        K[kK_W3T + ci * 128 + (26 - t) * 4 + co] = b;
    } else if (i < kP_B2) {
        Bk[i - kP_B1] = p;
    } else if (i < kP_B3) {
        Bk[32 + (i - kP_B2)] = p;
    } else {
        Bk[64 + (i - kP_B3)] = p;
    }
}

__global__ void k_dn_zero(float* __restrict__ p, int n, double* __restrict__ loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
    if (i == 0) *loss = 0.0;
}

__global__ void k_dn_zero_bf16(__bf16* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (__bf16)0.0f;
}

}  // namespace pic

using namespace pic;

namespace {

constexpr size_t kAl = 256;
size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

struct TrLayout {
    size_t P, M, V, G, K, Bk, loss, a1, a2, dy, dz2, dz1, y, g, t, total;
};

TrLayout tr_layout(const int32_t c[3]) {
    const size_t N = (size_t)c[0] * c[1] * c[2];
    TrLayout L;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = al(o + b);
        return at;
    };
    L.P = take(kP_N * 4);
    L.M = take(kP_N * 4);
    L.V = take(kP_N * 4);
    L.G = take(kG_N * 4);
    L.K = take(kK_N * 2);
    L.Bk = take(kB_N * 4);
    L.loss = take(8);
    L.a1 = take(N * 64);
    L.a2 = take(N * 64);
    L.dy = take(N * 8);
    L.dz2 = take(N * 64);
    L.dz1 = take(N * 64);
    L.y = take(N * 12);
    L.g = take(N * 12);
    L.t = take(N * 12);
    L.total = o;
    return L;
}

}  // namespace

struct pic_dn_trainer {
    int32_t n[3];
    hipStream_t st;
    char* ws;
    TrLayout L;
    float scale[3];
    double cell[3];
    int64_t steps = 0;
    bool has_params = false;
    bool train_bias = true;
    std::string err;
};

namespace {

pic_status tfail(pic_dn_trainer* t, pic_status s, const char* msg) {
    t->err = msg;
    return s;
}

#define THIPCHK(t, expr)                                                     \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess) {                                              \
            (t)->err = std::string(#expr) + ": " + hipGetErrorString(e_);    \
            return PIC_EDEVICE;                                              \
        }                                                                    \
    } while (0)

template <class T>
T* at(pic_dn_trainer* t, size_t off) {
    return reinterpret_cast<T*>(t->ws + off);
}

DnArgs base_args(pic_dn_trainer* t, float* const in[3], float* const target[3]) {
    DnArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.n[d] = t->n[d];
        a.bc[d] = 1;
        a.J[d] = in[d];
        a.Jt[d] = target ? target[d] : nullptr;
        a.scale[d] = t->scale[d];
        a.inv_scale[d] = 1.0f / t->scale[d];
    }
    a.origin = 0;
    a.loss = at<double>(t, t->L.loss);
    const double N = (double)t->n[0] * t->n[1] * t->n[2];
    a.grad_scale = (float)(2.0 / (3.0 * N));
    return a;
}

template <int CIN, int DC, int MB, bool INJ>
hipError_t wgrad(pic_dn_trainer* t, const WgArgs& w) {
    const size_t lds = (size_t)DN_HCELLS * CIN * 2 + (size_t)DN_TX * DN_TY * DN_TZ * DC * 2;
    hipError_t e = hipFuncSetAttribute((const void*)k_dn_wgrad<CIN, DC, MB, INJ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int grid = w.ntiles < 512 ? w.ntiles : 512;
    hipLaunchKernelGGL((k_dn_wgrad<CIN, DC, MB, INJ>), dim3(grid), dim3(DN_THREADS), lds, t->st, w);
    return hipGetLastError();
}

// Forward, loss and (unless forward_only) gradients of one crop (input,
// target: device FP32 SoA), added to the accumulated loss and gradient;
// `zero` clears them first.
pic_status tr_grad(pic_dn_trainer* t, float* const in[3], float* const target[3], bool zero = true,
                   bool forward_only = false) {
    const int ng = kG_N;
    if (zero) {
        hipLaunchKernelGGL(k_dn_zero, dim3((ng + 255) / 256), dim3(256), 0, t->st, at<float>(t, t->L.G), ng,
                           at<double>(t, t->L.loss));
        THIPCHK(t, hipGetLastError());
    }
    const __bf16* K = at<__bf16>(t, t->L.K);
    const float* Bk = at<float>(t, t->L.Bk);
    __bf16 *a1 = at<__bf16>(t, t->L.a1), *a2 = at<__bf16>(t, t->L.a2), *dy = at<__bf16>(t, t->L.dy);
    __bf16 *dz2 = at<__bf16>(t, t->L.dz2), *dz1 = at<__bf16>(t, t->L.dz1);
    float* G = at<float>(t, t->L.G);
    DnArgs a = base_args(t, in, target);
    // forward
    a.w = K + kK_W1, a.bias = Bk, a.act_out = a1;
    THIPCHK(t, launch_dn_layer(DN_L1_J_ACT, a, t->st));
    a.w = K + kK_W2, a.bias = Bk + 32, a.act_in = a1, a.act_out = a2;
    THIPCHK(t, launch_dn_layer(DN_L2_ACT, a, t->st));
    const size_t N = (size_t)t->n[0] * t->n[1] * t->n[2];
    float* y = at<float>(t, t->L.y);
    float* gJ = at<float>(t, t->L.g);
    a.w = K + kK_W3, a.bias = Bk + 64, a.act_in = a2, a.act_out = nullptr;
    for (int d = 0; d < 3; ++d) a.Jout[d] = y + d * N;
    THIPCHK(t, launch_dn_layer(DN_L3_Y, a, t->st));
    // t = J + sigma curl(y);  J' = B(t);  loss;  g = dL/dJ';  dy = sigma curl^T(B g)
    float* tb = at<float>(t, t->L.t);
    DnCombine c{};
    for (int d = 0; d < 3; ++d) {
        c.n[d] = t->n[d];
        c.bc[d] = 1;
        c.src[d] = in[d];
        c.y[d] = y + d * N;
        c.dst[d] = tb + d * N;
        c.T[d] = target[d];
        c.inv_scale[d] = 1.0f / t->scale[d];
        c.inv_d[d] = (float)(1.0 / t->cell[d]);
    }
    c.sigma = (float)(t->cell[0] * ((double)t->scale[0] + t->scale[1] + t->scale[2]) / 3.0);
    c.grad_scale = a.grad_scale;
    c.loss = a.loss;
    c.dy = dy;
    THIPCHK(t, launch_dn_curl_add(c, t->st));
    for (int d = 0; d < 3; ++d) {
        c.src[d] = tb + d * N;
        c.dst[d] = gJ + d * N;
    }
    THIPCHK(t, launch_dn_binomial(c, true, t->st));
    if (forward_only) return PIC_OK;
    for (int d = 0; d < 3; ++d) {
        c.src[d] = gJ + d * N;
        c.dst[d] = tb + d * N;
    }
    THIPCHK(t, launch_dn_binomial(c, false, t->st));     // B is symmetric: B^T g = B g
    for (int d = 0; d < 3; ++d) c.src[d] = tb + d * N;
    THIPCHK(t, launch_dn_curl_adjoint(c, t->st));
    // backward
    WgArgs w{};
    for (int d = 0; d < 3; ++d) {
        w.n[d] = t->n[d];
        w.bc[d] = 1;
        w.J[d] = in[d];
        w.inv_scale[d] = 1.0f / t->scale[d];
    }
    const dim3 gr = dn_grid(t->n);
    w.ntiles = (int)(gr.x * gr.y * gr.z);
    w.in = a2, w.dout = dy, w.dW = G + kG_W3, w.db = G + kG_B3;
    THIPCHK(t, (wgrad<32, 4, 1, false>(t, w)));
    a.c4_in = dy, a.w = K + kK_W3T, a.mask = a2, a.act_out = dz2;
    THIPCHK(t, launch_dn_layer(DN_L1_C4_MASK, a, t->st));
    w.in = a1, w.dout = dz2, w.dW = G + kG_W2, w.db = G + kG_B2;
    THIPCHK(t, (wgrad<32, 32, 2, false>(t, w)));
    a.act_in = dz2, a.w = K + kK_W2T, a.mask = a1, a.act_out = dz1;
    THIPCHK(t, launch_dn_layer(DN_L2_MASK, a, t->st));
    w.in = nullptr, w.dout = dz1, w.dW = G + kG_W1, w.db = G + kG_B1;
    THIPCHK(t, (wgrad<4, 32, 2, true>(t, w)));
    return PIC_OK;
}

pic_status tr_pack(pic_dn_trainer* t, float lr, float gscale = 1.0f) {
    float c1 = 1.0f, c2 = 1.0f;
    if (lr > 0.0f) {
        t->steps += 1;
        c1 = (float)(1.0 / (1.0 - pow(0.9, (double)t->steps)));
        c2 = (float)(1.0 / (1.0 - pow(0.999, (double)t->steps)));
    }
    hipLaunchKernelGGL(k_dn_adam_pack, dim3((kP_N + 255) / 256), dim3(256), 0, t->st, at<float>(t, t->L.P),
                       at<float>(t, t->L.M), at<float>(t, t->L.V), at<float>(t, t->L.G), at<__bf16>(t, t->L.K),
                       at<float>(t, t->L.Bk), lr, c1, c2, gscale, t->train_bias ? 1 : 0);
    THIPCHK(t, hipGetLastError());
    return PIC_OK;
}

bool valid_crop(const int32_t c[3]) {
    for (int d = 0; d < 3; ++d)
        if (c[d] < 1 || c[d] > 4096) return false;
    return (int64_t)c[0] * c[1] * c[2] < (1ll << 27);
}

}  // namespace

extern "C" {

size_t pic_dn_trainer_workspace_bytes(const int32_t crop[3]) {
    if (!crop || !valid_crop(crop)) return 0;
    return tr_layout(crop).total;
}

pic_status pic_dn_trainer_create(pic_dn_trainer** out, const int32_t crop[3], const double cell[3], void* workspace,
                                 size_t workspace_bytes, void* stream) {
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    if (!crop || !valid_crop(crop) || !cell || !workspace) return PIC_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!(cell[d] > 0.0) || !isfinite(cell[d])) return PIC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAl - 1)) != 0) return PIC_EINVAL;
    const TrLayout L = tr_layout(crop);
    if (workspace_bytes < L.total) return PIC_ENOMEM;
    pic_dn_trainer* t = new (std::nothrow) pic_dn_trainer();
    if (!t) return PIC_ENOMEM;
    for (int d = 0; d < 3; ++d) {
        t->n[d] = crop[d];
        t->scale[d] = 1.0f;
        t->cell[d] = cell[d];
    }
    t->st = reinterpret_cast<hipStream_t>(stream);
    t->ws = reinterpret_cast<char*>(workspace);
    t->L = L;
    // padding entries of the packed weights stay zero
    hipLaunchKernelGGL(k_dn_zero_bf16, dim3((kK_N + 255) / 256), dim3(256), 0, t->st, at<__bf16>(t, L.K), kK_N);
    if (hipGetLastError() != hipSuccess) {
        delete t;
        return PIC_EDEVICE;
    }
    *out = t;
    return PIC_OK;
}

pic_status pic_dn_trainer_set_params(pic_dn_trainer* t, const float* weights, const float* biases,
                                     const float* scale) {
    if (!t || !weights || !biases || !scale) return PIC_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!(scale[d] > 0.0f) || !isfinite(scale[d])) return tfail(t, PIC_EINVAL, "scales must be positive and finite");
    std::vector<float> p(kP_N);
    memcpy(p.data(), weights, sizeof(float) * kP_B1);
    memcpy(p.data() + kP_B1, biases, sizeof(float) * (kP_N - kP_B1));
    for (float v : p)
        if (!isfinite(v)) return tfail(t, PIC_EINVAL, "non-finite parameter");
    THIPCHK(t, hipMemcpyAsync(t->ws + t->L.P, p.data(), kP_N * 4, hipMemcpyHostToDevice, t->st));
    THIPCHK(t, hipMemsetAsync(t->ws + t->L.M, 0, kP_N * 4, t->st));
    THIPCHK(t, hipMemsetAsync(t->ws + t->L.V, 0, kP_N * 4, t->st));
    for (int d = 0; d < 3; ++d) t->scale[d] = scale[d];
    t->steps = 0;
    pic_status s = tr_pack(t, 0.0f);
    if (s != PIC_OK) return s;
    THIPCHK(t, hipStreamSynchronize(t->st));
    t->has_params = true;
    return PIC_OK;
}

pic_status pic_dn_trainer_get_params(pic_dn_trainer* t, float* weights, float* biases) {
    if (!t || !weights || !biases) return PIC_EINVAL;
    if (!t->has_params) return tfail(t, PIC_ESTATE, "parameters not set");
    std::vector<float> p(kP_N);
    THIPCHK(t, hipMemcpyAsync(p.data(), t->ws + t->L.P, kP_N * 4, hipMemcpyDeviceToHost, t->st));
    THIPCHK(t, hipStreamSynchronize(t->st));
    memcpy(weights, p.data(), sizeof(float) * kP_B1);
    memcpy(biases, p.data() + kP_B1, sizeof(float) * (kP_N - kP_B1));
    return PIC_OK;
}

pic_status pic_dn_trainer_step(pic_dn_trainer* t, float* const input[3], float* const target[3], float lr,
                               double* loss) {
    if (!t || !input || !target) return PIC_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!input[d] || !target[d]) return PIC_EINVAL;
    if (!t->has_params) return tfail(t, PIC_ESTATE, "parameters not set");
    if (!(lr > 0.0f) || !isfinite(lr)) return tfail(t, PIC_EINVAL, "learning rate must be positive");
    pic_status s = tr_grad(t, input, target);
    if (s != PIC_OK) return s;
    if (loss) {
        THIPCHK(t, hipMemcpyAsync(loss, t->ws + t->L.loss, 8, hipMemcpyDeviceToHost, t->st));
    }
    s = tr_pack(t, lr);
    if (s != PIC_OK) return s;
    if (loss) THIPCHK(t, hipStreamSynchronize(t->st));
    return PIC_OK;
}

pic_status pic_dn_trainer_step_batch(pic_dn_trainer* t, int32_t n, float* const* inputs, float* const* targets,
                                     float lr, double* loss) {
    if (!t || n < 1 || !inputs || !targets) return PIC_EINVAL;
    for (int32_t i = 0; i < 3 * n; ++i)
        if (!inputs[i] || !targets[i]) return PIC_EINVAL;
    if (!t->has_params) return tfail(t, PIC_ESTATE, "parameters not set");
    if (!(lr > 0.0f) || !isfinite(lr)) return tfail(t, PIC_EINVAL, "learning rate must be positive");
    for (int32_t i = 0; i < n; ++i) {
        pic_status s = tr_grad(t, inputs + 3 * i, targets + 3 * i, i == 0);
        if (s != PIC_OK) return s;
    }
    if (loss) THIPCHK(t, hipMemcpyAsync(loss, t->ws + t->L.loss, 8, hipMemcpyDeviceToHost, t->st));
    pic_status s = tr_pack(t, lr, 1.0f / (float)n);
    if (s != PIC_OK) return s;
    if (loss) {
        THIPCHK(t, hipStreamSynchronize(t->st));
        *loss /= (double)n;
    }
    return PIC_OK;
}

pic_status pic_dn_trainer_eval(pic_dn_trainer* t, int32_t n, float* const* inputs, float* const* targets,
                               double* loss) {
    if (!t || n < 1 || !inputs || !targets || !loss) return PIC_EINVAL;
    for (int32_t i = 0; i < 3 * n; ++i)
        if (!inputs[i] || !targets[i]) return PIC_EINVAL;
    if (!t->has_params) return tfail(t, PIC_ESTATE, "parameters not set");
    for (int32_t i = 0; i < n; ++i) {
        pic_status s = tr_grad(t, inputs + 3 * i, targets + 3 * i, i == 0, true);
        if (s != PIC_OK) return s;
    }
    THIPCHK(t, hipMemcpyAsync(loss, t->ws + t->L.loss, 8, hipMemcpyDeviceToHost, t->st));
    THIPCHK(t, hipStreamSynchronize(t->st));
    *loss /= (double)n;
    return PIC_OK;
}

pic_status pic_dn_trainer_grad(pic_dn_trainer* t, float* const input[3], float* const target[3], double* loss,
                               float* grad_weights, float* grad_biases) {
    if (!t || !input || !target || !loss || !grad_weights || !grad_biases) return PIC_EINVAL;
    if (!t->has_params) return tfail(t, PIC_ESTATE, "parameters not set");
    pic_status s = tr_grad(t, input, target);
    if (s != PIC_OK) return s;
    std::vector<float> g(kG_N);
    THIPCHK(t, hipMemcpyAsync(g.data(), t->ws + t->L.G, kG_N * 4, hipMemcpyDeviceToHost, t->st));
    THIPCHK(t, hipMemcpyAsync(loss, t->ws + t->L.loss, 8, hipMemcpyDeviceToHost, t->st));
    THIPCHK(t, hipStreamSynchronize(t->st));
    for (int co = 0; co < 32; ++co)
        for (int ci = 0; ci < 3; ++ci)
            for (int tp = 0; tp < 27; ++tp) grad_weights[kP_W1 + (co * 3 + ci) * 27 + tp] = g[kG_W1 + co * 112 + tp * 4 + ci];
    for (int co = 0; co < 32; ++co)
        for (int ci = 0; ci < 32; ++ci)
            for (int tp = 0; tp < 27; ++tp)
                grad_weights[kP_W2 + (co * 32 + ci) * 27 + tp] = g[kG_W2 + co * 864 + tp * 32 + ci];
    for (int co = 0; co < 3; ++co)
        for (int ci = 0; ci < 32; ++ci)
            for (int tp = 0; tp < 27; ++tp)
                grad_weights[kP_W3 + (co * 32 + ci) * 27 + tp] = g[kG_W3 + co * 864 + tp * 32 + ci];
    for (int i = 0; i < 32; ++i) grad_biases[i] = g[kG_B1 + i];
    for (int i = 0; i < 32; ++i) grad_biases[32 + i] = g[kG_B2 + i];
    for (int i = 0; i < 3; ++i) grad_biases[64 + i] = g[kG_B3 + i];
    return PIC_OK;
}

pic_status pic_dn_trainer_freeze_biases(pic_dn_trainer* t, int32_t freeze) {
    if (!t) return PIC_EINVAL;
    t->train_bias = freeze == 0;
    return PIC_OK;
}

const char* pic_dn_trainer_last_error(const pic_dn_trainer* t) {
    if (!t) return "null trainer";
    return t->err.c_str();
}

void pic_dn_trainer_destroy(pic_dn_trainer* t) {
    if (!t) return;
    (void)hipStreamSynchronize(t->st);
    delete t;
}

}  // extern "C"
