// Learned current denoiser: three 3x3x3 convolution layers on the deposited
// current, as implicit GEMMs on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation).
//
//   x  = bf16(J_d / s_d)                    layer 1: 3 (padded to 4) -> 32 channels
//   a1 = bf16(relu(conv(x, W1) + b1))
//   a2 = bf16(relu(conv(a1, W2) + b2))      layer 2: 32 -> 32 (84 % of the work)
//   J'_d = J_d + s_d (conv(a2, W3) + b3)_d  layer 3: 32 -> 3 (padded to 16)
//
// conv is the "same"-size 3x3x3 cross-correlation; y and z are periodic, x is
// periodic or (moving window) zero beyond the window's two ends, or zero
// outside the box on any axis (training crops).  Activations live in HBM
// channels-last as bf16 [cell][32] (64 B per cell).
//
// One workgroup of 8 wavefronts computes a tile of 16 x 4 x 8 cells (x, y, z)
// in window coordinates: it stages the tile's input halo (18 x 6 x 10 cells,
// rows padded to 20) and the layer's weights in LDS, then each wavefront
// takes one z-plane: 4 rows of 16 cells = 4 MFMA row blocks, times 2 (or 1)
// blocks of 16 output channels, accumulated over the 27 taps x 32 input
// channels (one MFMA K-step of 32 per tap).
//
// MFMA operand layout (16x16x32): lane l holds A row l%16, K elements
// 8(l/16)..8(l/16)+7; B column l%16 with the same K elements; the result
// holds column l%16, rows 4(l/16)..4(l/16)+3.  A row = a cell, K = input
// channels, B column = an output channel.
//
// LDS rows of 64 B (a cell's 32 channels, or a weight row) are stored as four
// 16-byte chunks rotated by rot(r) = ((r >> 1) ^ (r >> 2)) & 3, so that the 16
// consecutive rows one A or B read touches spread over all banks.
#include "pic_internal.h"

namespace pic {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DN_TX = 16, DN_TY = 4, DN_TZ = 8;        // output tile
constexpr int DN_HX = 20, DN_HY = DN_TY + 2, DN_HZ = DN_TZ + 2;   // halo tile (x padded)
constexpr int DN_HCELLS = DN_HX * DN_HY * DN_HZ;
constexpr int DN_THREADS = 512;

__device__ __forceinline__ int dn_rot(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// Byte offset of 16-byte chunk q of 64-byte row r.
__device__ __forceinline__ int dn_chunk(int r, int q) { return r * 64 + (((q + dn_rot(r)) & 3) << 4); }

// Storage index along one axis of window/box coordinate v, or -1 when the
// neighbour reads as zero.  bc: 0 periodic, 1 zero outside [0, n), 2 moving
// window (zero outside [0, n), storage = (v + origin) mod n).
__device__ __forceinline__ int dn_axis(int v, int n, int bc, int origin) {
    if (bc == 0) return v < 0 ? v + n : (v >= n ? v - n : v);
    if (v < 0 || v >= n) return -1;
    if (bc == 2) {
        v += origin;
        return v >= n ? v - n : v;
    }
    return v;
}

struct DnArgs {
    int n[3];
    int bc[3];
    int origin;
    const float* J[3];        // layer 1 input; layer 3 residual input
    float* Jout[3];           // layer 3 output
    const __bf16* act_in;     // layers 2, 3 input [cell][32]
    __bf16* act_out;          // layers 1, 2 output [cell][32]
    const __bf16* w;          // packed weights (see the host packing)
    const float* bias;
    float scale[3], inv_scale[3];
};

// Tile origin (window coordinates) of this workgroup.
__device__ __forceinline__ void dn_tile(int t0[3]) {
    t0[0] = blockIdx.x * DN_TX;
    t0[1] = blockIdx.y * DN_TY;
    t0[2] = blockIdx.z * DN_TZ;
}

// Copy `rows` 64-byte rows of packed weights into LDS (swizzled).
__device__ __forceinline__ void dn_stage_weights(const __bf16* __restrict__ w, int rows, char* lds) {
    const uint4* src = reinterpret_cast<const uint4*>(w);
    for (int g = threadIdx.x; g < rows * 4; g += DN_THREADS)
        *reinterpret_cast<uint4*>(lds + dn_chunk(g >> 2, g & 3)) = src[g];
}

// Storage cell index of halo cell (hx, hy, hz) of the tile, or -1 for zero.
__device__ __forceinline__ int dn_halo_src(const DnArgs& a, const int t0[3], int hx, int hy, int hz) {
    const int x = dn_axis(t0[0] - 1 + hx, a.n[0], a.bc[0], a.origin);
    const int y = dn_axis(t0[1] - 1 + hy, a.n[1], a.bc[1], 0);
    const int z = dn_axis(t0[2] - 1 + hz, a.n[2], a.bc[2], 0);
    if (x < 0 || y < 0 || z < 0) return -1;
    return x + a.n[0] * (y + a.n[1] * z);
}

// Stage a 32-channel bf16 activation halo.
__device__ __forceinline__ void dn_stage_act(const DnArgs& a, const int t0[3], char* lds) {
    const uint4* src = reinterpret_cast<const uint4*>(a.act_in);
    for (int g = threadIdx.x; g < DN_HCELLS * 4; g += DN_THREADS) {
        const int c = g >> 2, q = g & 3;
        const int hx = c % DN_HX, r = c / DN_HX, hy = r % DN_HY, hz = r / DN_HY;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (hx < DN_TX + 2) {
            const int s = dn_halo_src(a, t0, hx, hy, hz);
            if (s >= 0) v = src[(size_t)s * 4 + q];
        }
        *reinterpret_cast<uint4*>(lds + dn_chunk(c, q)) = v;
    }
}

// Storage cell of output row block `blk` (y row), lane row m, plane lz; -1 outside the box.
__device__ __forceinline__ int dn_out_cell(const DnArgs& a, const int t0[3], int lz, int blk, int m) {
    const int x = t0[0] + m, y = t0[1] + blk, z = t0[2] + lz;
    if (x >= a.n[0] || y >= a.n[1] || z >= a.n[2]) return -1;
    const int xs = a.bc[0] == 2 ? (x + a.origin >= a.n[0] ? x + a.origin - a.n[0] : x + a.origin) : x;
    return xs + a.n[0] * (y + a.n[1] * z);
}

// Accumulate the 27 taps x 32 input channels of a 32-channel layer.
template <int NH>
__device__ __forceinline__ void dn_mma32(const char* act, const char* wl, f32x4 acc[4][NH]) {
    const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int m = l & 15, q = l >> 4;
#pragma unroll 1
    for (int tap = 0; tap < 27; ++tap) {
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // 0..2 = offset + 1
        bf16x8 B[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h)
            B[h] = *reinterpret_cast<const bf16x8*>(wl + dn_chunk(tap * 16 * NH + h * 16 + m, q));
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            const int c = ((lz + dz) * DN_HY + (blk + dy)) * DN_HX + (m + dx);
            const bf16x8 A = *reinterpret_cast<const bf16x8*>(act + dn_chunk(c, q));
#pragma unroll
            for (int h = 0; h < NH; ++h) acc[blk][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[h], acc[blk][h], 0, 0, 0);
        }
    }
}

// bf16 relu(acc + bias) into the channels-last output.
__device__ __forceinline__ void dn_store_act(const DnArgs& a, const int t0[3], const f32x4 acc[4][2]) {
    const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int col = l & 15, rq = l >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int co = h * 16 + col;
        const float b = a.bias[co];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int cell = dn_out_cell(a, t0, lz, blk, rq * 4 + j);
                if (cell < 0) continue;
                const float v = fmaxf(acc[blk][h][j] + b, 0.0f);
                a.act_out[(size_t)cell * 32 + co] = (__bf16)v;
            }
    }
}

// Layer 1: J (3 x FP32) -> 32 channels.  K = tap * 4 + channel (channel 3 and
// taps 27..31 are zero), 4 K-steps of 32; lane chunk q of step s covers taps
// 8s + 2q and 8s + 2q + 1.
__global__ void __launch_bounds__(DN_THREADS) k_dn_layer1(DnArgs a) {
    __shared__ __attribute__((aligned(16))) char lds[DN_HCELLS * 8 + 32 * 256];
    char* xin = lds;                       // [halo cell][4] bf16
    char* wl = lds + DN_HCELLS * 8;        // [co][128] bf16, 256 B rows (4 chunks of 64 B)
    int t0[3];
    dn_tile(t0);
    {   // weights: 32 rows of 256 B, plain order
        const uint4* src = reinterpret_cast<const uint4*>(a.w);
        for (int g = threadIdx.x; g < 32 * 16; g += DN_THREADS) reinterpret_cast<uint4*>(wl)[g] = src[g];
    }
    for (int c = threadIdx.x; c < DN_HCELLS; c += DN_THREADS) {
        const int hx = c % DN_HX, r = c / DN_HX, hy = r % DN_HY, hz = r / DN_HY;
        bf16x4 v = {(__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
        if (hx < DN_TX + 2) {
            const int s = dn_halo_src(a, t0, hx, hy, hz);
            if (s >= 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) v[d] = (__bf16)(a.J[d][s] * a.inv_scale[d]);
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
            for (int h = 0; h < 2; ++h) acc[blk][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[h], acc[blk][h], 0, 0, 0);
        }
    }
    dn_store_act(a, t0, acc);
}

// Layer 2: 32 -> 32 channels.
__global__ void __launch_bounds__(DN_THREADS) k_dn_layer2(DnArgs a) {
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
    dn_store_act(a, t0, acc);
}

// Layer 3: 32 -> 3 channels (16 computed), residual into J'.
__global__ void __launch_bounds__(DN_THREADS) k_dn_layer3(DnArgs a) {
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
    if (co >= 3) return;
    const float b = a.bias[co], s = a.scale[co];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cell = dn_out_cell(a, t0, lz, blk, rq * 4 + j);
            if (cell < 0) continue;
            a.Jout[co][cell] = fmaf(s, acc[blk][0][j] + b, a.J[co][cell]);
        }
}

size_t denoise_lds_bytes(int layer) {
    if (layer == 2) return (size_t)DN_HCELLS * 64 + 27 * 32 * 64;
    if (layer == 3) return (size_t)DN_HCELLS * 64 + 27 * 16 * 64;
    return 0;
}

hipError_t launch_denoise(const Geom& g, const int bc[3], const DenoiseWeights& w, float* const Jin[3],
                          float* const Jout[3], __bf16* h1, __bf16* h2, hipStream_t st) {
    DnArgs a;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bc[d] = bc[d];
        a.J[d] = Jin[d];
        a.Jout[d] = Jout[d];
        a.scale[d] = w.scale[d];
        a.inv_scale[d] = 1.0f / w.scale[d];
    }
    a.origin = g.window ? g.origin : 0;
    const dim3 grid((g.n[0] + DN_TX - 1) / DN_TX, (g.n[1] + DN_TY - 1) / DN_TY, (g.n[2] + DN_TZ - 1) / DN_TZ);
    const size_t l2 = denoise_lds_bytes(2), l3 = denoise_lds_bytes(3);
    hipError_t e = hipFuncSetAttribute((const void*)k_dn_layer2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_dn_layer3, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l3);
    if (e != hipSuccess) return e;
    a.act_in = nullptr;
    a.act_out = h1;
    a.w = w.w1;
    a.bias = w.b1;
    hipLaunchKernelGGL(k_dn_layer1, grid, dim3(DN_THREADS), 0, st, a);
    a.act_in = h1;
    a.act_out = h2;
    a.w = w.w2;
    a.bias = w.b2;
    hipLaunchKernelGGL(k_dn_layer2, grid, dim3(DN_THREADS), l2, st, a);
    a.act_in = h2;
    a.act_out = nullptr;
    a.w = w.w3;
    a.bias = w.b3;
    hipLaunchKernelGGL(k_dn_layer3, grid, dim3(DN_THREADS), l3, st, a);
    return hipGetLastError();
}

}  // namespace pic
