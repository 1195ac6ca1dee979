// Learned current denoiser: the convolution layers of the network described
// in pic_dn_common.h.  Inference runs layers 1, 2, 3 with the relu and
// residual epilogues; training reuses the same layer shapes for the gradient
// of the loss with respect to the activations (a transposed convolution is a
// convolution with the taps mirrored and the channel roles swapped), with a
// relu-mask epilogue, and a layer-3 epilogue that forms the loss.
#include "pic_dn_common.h"

namespace pic {

// 32 output channels: EPI 0 = bf16 relu(acc + bias), 1 = bf16 acc where the mask activation is > 0.
template <int EPI>
__device__ __forceinline__ void dn_store32(const DnArgs& a, const int t0[3], const f32x4 acc[4][2]) {
    const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int col = l & 15, rq = l >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int co = h * 16 + col;
        const float b = EPI == 0 ? a.bias[co] : 0.0f;
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int cell = dn_out_cell(a, t0, lz, blk, rq * 4 + j);
                if (cell < 0) continue;
                float v;
                if (EPI == 0)
                    v = fmaxf(acc[blk][h][j] + b, 0.0f);
                else
                    v = (float)a.mask[(size_t)cell * 32 + co] > 0.0f ? acc[blk][h][j] : 0.0f;
                a.act_out[(size_t)cell * 32 + co] = (__bf16)v;
            }
    }
}

// 4-channel input (3 used), 32 output channels.  K = tap * 4 + channel
// (channel 3 and taps 27..31 zero), 4 K-steps of 32; lane chunk q of step s
// covers taps 8s + 2q and 8s + 2q + 1.  IN 0: the current J_d / s_d (FP32,
// rounded to bf16 here); IN 1: a bf16 [cell][4] array.
template <int IN, int EPI>
__global__ void __launch_bounds__(DN_THREADS) k_dn_c4(DnArgs a) {
    __shared__ __attribute__((aligned(16))) char lds[DN_HCELLS * 8 + 32 * 256];
    char* xin = lds;                       // [halo cell][4] bf16
    char* wl = lds + DN_HCELLS * 8;        // [co][128] bf16, 256 B rows
    int t0[3];
    dn_tile(t0);
    {
        const uint4* src = reinterpret_cast<const uint4*>(a.w);
        for (int g = threadIdx.x; g < 32 * 16; g += DN_THREADS) reinterpret_cast<uint4*>(wl)[g] = src[g];
    }
    for (int c = threadIdx.x; c < DN_HCELLS; c += DN_THREADS) {
        const int hx = c % DN_HX, r = c / DN_HX, hy = r % DN_HY, hz = r / DN_HY;
        bf16x4 v = {(__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
        if (hx < DN_TX + 2) {
            const int s = dn_halo_src(a, t0, hx, hy, hz);
            if (s >= 0) {
                if (IN == 0) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) v[d] = (__bf16)(a.J[d][s] * a.inv_scale[d]);
                } else {
                    v = reinterpret_cast<const bf16x4*>(a.c4_in)[s];
                }
            }
        }
        *reinterpret_cast<bf16x4*>(xin + c * 8) = v;
    }
    __syncthreads();
    const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int m = l & 15, q = l >> 4;
    f32x4 acc[4][2];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[blk][h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        bf16x8 B[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
            B[h] = *reinterpret_cast<const bf16x8*>(wl + (h * 16 + m) * 256 + s * 64 + q * 16);
        const int ta = 8 * s + 2 * q;
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            bf16x8 A;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int tap = ta + half;
                bf16x4 v = {(__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
                if (tap < 27) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    const int c = ((lz + dz) * DN_HY + (blk + dy)) * DN_HX + (m + dx);
                    v = *reinterpret_cast<const bf16x4*>(xin + c * 8);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) A[half * 4 + e] = v[e];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
                acc[blk][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[h], acc[blk][h], 0, 0, 0);
        }
    }
    dn_store32<EPI>(a, t0, acc);
}

// 32 -> 32 channels.
template <int EPI>
__global__ void __launch_bounds__(DN_THREADS) k_dn_c32(DnArgs a) {
    extern __shared__ __attribute__((aligned(16))) char dlds[];
    char* act = dlds;
    char* wl = dlds + DN_HCELLS * 64;
    int t0[3];
    dn_tile(t0);
    dn_stage_weights(a.w, 27 * 32, wl);
    dn_stage_act(a, t0, act);
    __syncthreads();
    f32x4 acc[4][2];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[blk][h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    dn_mma32<2>(act, wl, acc);
    dn_store32<EPI>(a, t0, acc);
}

// 32 -> 3 channels (16 computed).  EPI 0: residual J' = J + s (acc + b);
// EPI 1: loss of y = acc + b against r = (J_target - J) / s, and its
// gradient 2 (y - r) / (3 N) as bf16 [cell][4] (channel 3 zero).
template <int EPI>
__global__ void __launch_bounds__(DN_THREADS) k_dn_c3(DnArgs a) {
    extern __shared__ __attribute__((aligned(16))) char dlds[];
    char* act = dlds;
    char* wl = dlds + DN_HCELLS * 64;
    int t0[3];
    dn_tile(t0);
    dn_stage_weights(a.w, 27 * 16, wl);
    dn_stage_act(a, t0, act);
    __syncthreads();
    f32x4 acc[4][1];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) acc[blk][0] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    dn_mma32<1>(act, wl, acc);
    const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int co = l & 15, rq = l >> 4;
    if (co > 3 || (EPI == 0 && co == 3)) return;
    double part = 0.0;
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cell = dn_out_cell(a, t0, lz, blk, rq * 4 + j);
            if (cell < 0) continue;
            if (EPI == 0) {
                a.Jout[co][cell] = fmaf(a.scale[co], acc[blk][0][j] + a.bias[co], a.J[co][cell]);
            } else if (co == 3) {
                a.c4_out[(size_t)cell * 4 + 3] = (__bf16)0.0f;
            } else {
                const float y = acc[blk][0][j] + a.bias[co];
                const float r = (a.Jt[co][cell] - a.J[co][cell]) * a.inv_scale[co];
                const float e = y - r;
                part += (double)e * (double)e;
                a.c4_out[(size_t)cell * 4 + co] = (__bf16)(a.grad_scale * e);
            }
        }
    if (EPI == 1 && co < 3) atomicAdd(a.loss, part * (0.5 * (double)a.grad_scale));
}

static size_t dn_lds(int cout) { return (size_t)DN_HCELLS * 64 + (size_t)27 * cout * 64; }

template <class K>
static hipError_t dn_launch(K kern, size_t lds, const DnArgs& a, hipStream_t st) {
    if (lds > 0) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dn_grid(a.n), dim3(DN_THREADS), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dn_layer(int kind, const DnArgs& a, hipStream_t st) {
    switch (kind) {
        case DN_L1_J_ACT: return dn_launch(k_dn_c4<0, 0>, 0, a, st);
        case DN_L1_C4_MASK: return dn_launch(k_dn_c4<1, 1>, 0, a, st);
        case DN_L2_ACT: return dn_launch(k_dn_c32<0>, dn_lds(32), a, st);
        case DN_L2_MASK: return dn_launch(k_dn_c32<1>, dn_lds(32), a, st);
        case DN_L3_RESID: return dn_launch(k_dn_c3<0>, dn_lds(16), a, st);
        case DN_L3_LOSS: return dn_launch(k_dn_c3<1>, dn_lds(16), a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_denoise(const Geom& g, const int bc[3], const DenoiseWeights& w, float* const Jin[3],
                          float* const Jout[3], __bf16* h1, __bf16* h2, hipStream_t st) {
    DnArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bc[d] = bc[d];
        a.J[d] = Jin[d];
        a.Jout[d] = Jout[d];
        a.scale[d] = w.scale[d];
        a.inv_scale[d] = 1.0f / w.scale[d];
    }
    a.origin = g.window ? g.origin : 0;
    a.act_out = h1;
    a.w = w.w1;
    a.bias = w.b1;
    hipError_t e = launch_dn_layer(DN_L1_J_ACT, a, st);
    if (e != hipSuccess) return e;
    a.act_in = h1;
    a.act_out = h2;
    a.w = w.w2;
    a.bias = w.b2;
    e = launch_dn_layer(DN_L2_ACT, a, st);
    if (e != hipSuccess) return e;
    a.act_in = h2;
    a.act_out = nullptr;
    a.w = w.w3;
    a.bias = w.b3;
    return launch_dn_layer(DN_L3_RESID, a, st);
}

}  // namespace pic
