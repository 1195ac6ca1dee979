// Building blocks of the learned current denoiser's convolutions (inference
// and training): three 3x3x3 convolution layers on the deposited current, as
// implicit GEMMs on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation).
//
//   x  = bf16(J_d / s_d)                    layer 1: 3 (padded to 4) -> 32 channels
//   a1 = bf16(relu(conv(x, W1) + b1))
//   a2 = bf16(relu(conv(a1, W2) + b2))      layer 2: 32 -> 32 (84 % of the work)
//   J'_d = J_d + s_d (conv(a2, W3) + b3)_d  layer 3: 32 -> 3 (4 row blocks x 4 columns)
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
// Weight rows of 64 B are stored in LDS as four 16-byte chunks rotated by
// rot(r) = ((r >> 1) ^ (r >> 2)) & 3, so that the consecutive rows one B read
// touches spread over all banks; rot(r + 16 k) = rot(r), so the rows of every
// tap are the first 16 rows moved by a constant.  The input halo's cell rows
// are padded to 80 B instead (8 consecutive cells, one 16-byte read each,
// fall in disjoint bank quadruples), so every A read of a wavefront is one
// base address plus a constant per tap.
#pragma once

#include "pic_internal.h"

namespace pic {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DN_TX = 16, DN_TY = 4, DN_TZ = 8;        // output tile
constexpr int DN_HX = 20, DN_HY = DN_TY + 2, DN_HZ = DN_TZ + 2;   // halo tile (x padded)
constexpr int DN_HCELLS = DN_HX * DN_HY * DN_HZ;
constexpr int DN_THREADS = 512;
constexpr int DN_ROWB = 80;                               // LDS bytes per halo cell row
constexpr int DN_ACT_LDS = DN_HCELLS * DN_ROWB;

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
    const __bf16* act_in;     // 32-channel input [cell][32]
    __bf16* act_out;          // 32-channel output [cell][32]
    const __bf16* w;          // packed weights (see the host packing)
    const float* bias;
    float scale[3], inv_scale[3];
    // training
    const __bf16* c4_in;      // 4-channel input [cell][4] (output gradient of layer 3)
    const __bf16* mask;       // relu mask source [cell][32] (an activation: > 0 passes)
    const float* Jt[3];       // target current
    __bf16* c4_out;           // 4-channel output [cell][4] (loss gradient of y)
    double* loss;             // += sum of squared errors / (3 N)
    float grad_scale;         // 2 / (3 N)
};

// Kernel variants: input of the 4-channel-input shape, and epilogues.
// DN_L3_Y writes y = conv(a2, W3) + b3 as FP32 components into Jout.
enum { DN_L1_J_ACT = 0, DN_L1_C4_MASK, DN_L2_ACT, DN_L2_MASK, DN_L3_Y };

// Output stage J' = B(J + sigma curl(y)) (backward-difference curl, binomial
// filter B), and for training the loss against a target and the gradient.
struct DnCombine {
    int n[3];
    int bc[3];
    int origin;
    const float* src[3];    // curl_add: J;   binomial: its input
    const float* y[3];
    float* dst[3];          // curl_add: J + sigma curl(y);  binomial: B(src) (or the loss gradient)
    float sigma;
    float inv_d[3];
    // training
    const float* T[3];
    float inv_scale[3];
    float grad_scale;       // 2 / (3 N)
    double* loss;
    __bf16* dy;             // sigma curl^T(src) as bf16 [cell][4]
};

// dst = src + sigma curl(y)
hipError_t launch_dn_curl_add(const DnCombine& c, hipStream_t st);
// dst = B(src); with loss: J' = B(src) against T, dst = dL/dJ' = grad_scale (J' - T) / s^2
hipError_t launch_dn_binomial(const DnCombine& c, bool loss, hipStream_t st);
// dy = sigma curl^T(src)
hipError_t launch_dn_curl_adjoint(const DnCombine& c, hipStream_t st);

// Output tiles of a box of n cells.
inline dim3 dn_grid(const int n[3]) {
    return dim3((n[0] + DN_TX - 1) / DN_TX, (n[1] + DN_TY - 1) / DN_TY, (n[2] + DN_TZ - 1) / DN_TZ);
}

hipError_t launch_dn_layer(int kind, const DnArgs& a, hipStream_t st);

// Tile origin (window coordinates) of this workgroup.
__device__ __forceinline__ void dn_tile(int t0[3]) {
    t0[0] = blockIdx.x * DN_TX;
    t0[1] = blockIdx.y * DN_TY;
    t0[2] = blockIdx.z * DN_TZ;
}

// Copy ROWS 64-byte rows of packed weights into LDS (swizzled).  Each thread
// issues all its global loads before its first LDS store, so the staging
// waits for one memory latency rather than one per chunk.
template <int ROWS>
__device__ __forceinline__ void dn_stage_weights(const __bf16* __restrict__ w, char* lds) {
    constexpr int N = ROWS * 4, PER = (N + DN_THREADS - 1) / DN_THREADS;
    const uint4* src = reinterpret_cast<const uint4*>(w);
    uint4 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int g = threadIdx.x + k * DN_THREADS;
        v[k] = make_uint4(0u, 0u, 0u, 0u);
        if (g < N) v[k] = src[g];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int g = threadIdx.x + k * DN_THREADS;
        if (g < N) *reinterpret_cast<uint4*>(lds + dn_chunk(g >> 2, g & 3)) = v[k];
    }
}

// Storage cell index of halo cell (hx, hy, hz) of the tile, or -1 for zero.
__device__ __forceinline__ int dn_halo_src(const DnArgs& a, const int t0[3], int hx, int hy, int hz) {
    const int x = dn_axis(t0[0] - 1 + hx, a.n[0], a.bc[0], a.origin);
    const int y = dn_axis(t0[1] - 1 + hy, a.n[1], a.bc[1], 0);
    const int z = dn_axis(t0[2] - 1 + hz, a.n[2], a.bc[2], 0);
    if (x < 0 || y < 0 || z < 0) return -1;
    return x + a.n[0] * (y + a.n[1] * z);
}

// A 32-channel bf16 activation halo in two phases: every global load of the
// thread into registers (they can stay in flight while the previous tile's
// matrix work runs), then the LDS stores.  The halo coordinates of the
// thread's chunks do not depend on the tile: dn_halo_coords packs them once
// (hx | hy << 8 | hz << 16 | chunk << 24, or -1 for no load).
constexpr int DN_ACT_PER = (DN_HCELLS * 4 + DN_THREADS - 1) / DN_THREADS;

__device__ __forceinline__ void dn_halo_coords(int hc[DN_ACT_PER]) {
#pragma unroll
    for (int k = 0; k < DN_ACT_PER; ++k) {
        const int g = threadIdx.x + k * DN_THREADS;
        const int c = g >> 2, q = g & 3;
        const int hx = c % DN_HX, r = c / DN_HX, hy = r % DN_HY, hz = r / DN_HY;
        hc[k] = g < DN_HCELLS * 4 && hx < DN_TX + 2 ? hx | (hy << 8) | (hz << 16) | (q << 24) : -1;
    }
}

// Grid and boundary of a layer held in registers for the halo loads.
struct DnBox {
    int n[3], bc[3], origin;
};

__device__ __forceinline__ DnBox dn_box(const DnArgs& a) {
    DnBox b;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        b.n[d] = a.n[d];
        b.bc[d] = a.bc[d];
    }
    b.origin = a.origin;
    return b;
}

// dn_axis for v in [-1, n] without branches (v one cell beyond the box at most).
__device__ __forceinline__ int dn_axis_sel(int v, int n, int bc, int origin) {
    const bool out = v < 0 || v >= n;
    const int w = v < 0 ? v + n : (v >= n ? v - n : v);
    int x = v + origin;
    x = x >= n ? x - n : x;
    const int r = bc == 0 ? w : (bc == 2 ? x : v);
    return bc != 0 && out ? -1 : r;
}

__device__ __forceinline__ void dn_load_act(const DnArgs& a, const DnBox& b, const int t0[3],
                                            const int hc[DN_ACT_PER], uint4 v[DN_ACT_PER]) {
    const uint4* src = reinterpret_cast<const uint4*>(a.act_in);
    long long off[DN_ACT_PER];
#pragma unroll
    for (int k = 0; k < DN_ACT_PER; ++k) {
        const int x = dn_axis_sel(t0[0] - 1 + (hc[k] & 255), b.n[0], b.bc[0], b.origin);
        const int y = dn_axis_sel(t0[1] - 1 + ((hc[k] >> 8) & 255), b.n[1], b.bc[1], 0);
        const int z = dn_axis_sel(t0[2] - 1 + ((hc[k] >> 16) & 255), b.n[2], b.bc[2], 0);
        const bool ok = hc[k] >= 0 && x >= 0 && y >= 0 && z >= 0;
        off[k] = ok ? ((long long)x + (long long)b.n[0] * (y + (long long)b.n[1] * z)) * 4 + (hc[k] >> 24) : -1;
    }
#pragma unroll
    for (int k = 0; k < DN_ACT_PER; ++k) v[k] = off[k] >= 0 ? src[off[k]] : make_uint4(0u, 0u, 0u, 0u);
}

__device__ __forceinline__ void dn_store_act(const uint4 v[DN_ACT_PER], char* lds) {
    constexpr int N = DN_HCELLS * 4;
#pragma unroll
    for (int k = 0; k < DN_ACT_PER; ++k) {
        const int g = threadIdx.x + k * DN_THREADS;
        if (g < N) *reinterpret_cast<uint4*>(lds + (g >> 2) * DN_ROWB + (g & 3) * 16) = v[k];
    }
}

// Output tiles of the box and the origin of tile t (x fastest).
__device__ __forceinline__ int dn_ntiles(const int n[3], int* ntx, int* nty) {
    *ntx = (n[0] + DN_TX - 1) / DN_TX;
    *nty = (n[1] + DN_TY - 1) / DN_TY;
    return *ntx * *nty * ((n[2] + DN_TZ - 1) / DN_TZ);
}

__device__ __forceinline__ void dn_tile_of(int t, int ntx, int nty, int t0[3]) {
    const int bx = t % ntx, r = t / ntx;
    t0[0] = bx * DN_TX;
    t0[1] = (r % nty) * DN_TY;
    t0[2] = (r / nty) * DN_TZ;
}

// Storage cell of output row block `blk` (y row), lane row m, plane lz; -1 outside the box.
__device__ __forceinline__ int dn_out_cell(const DnArgs& a, const int t0[3], int lz, int blk, int m) {
    const int x = t0[0] + m, y = t0[1] + blk, z = t0[2] + lz;
    if (x >= a.n[0] || y >= a.n[1] || z >= a.n[2]) return -1;
    const int xs = a.bc[0] == 2 ? (x + a.origin >= a.n[0] ? x + a.origin - a.n[0] : x + a.origin) : x;
    return xs + a.n[0] * (y + a.n[1] * z);
}

// Accumulate the 27 taps x 32 input channels of a 32-channel layer.  Per tap
// column (dz, dx) the wavefront reads the 6 halo rows its 4 output rows need
// once and reuses each for the three dy taps (row blk + dy): 6 A reads per 12
// row-block MFMA steps.  All taps are unrolled, so every LDS address is the
// lane's base plus a constant.
template <int NH>
__device__ __forceinline__ void dn_mma32(const char* act, const char* wl, f32x4 acc[4][NH]) {
    const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int m = l & 15, q = l >> 4;
    const char* abase = act + (lz * DN_HY * DN_HX + m) * DN_ROWB + q * 16;
    const char* bbase = wl + dn_chunk(m, q);
#pragma unroll
    for (int zx = 0; zx < 9; ++zx) {
        const int dz = zx / 3, dx = zx % 3;   // 0..2 = offset + 1
        bf16x8 A[DN_HY];
#pragma unroll
        for (int r = 0; r < DN_HY; ++r)
            A[r] = *reinterpret_cast<const bf16x8*>(abase + ((dz * DN_HY + r) * DN_HX + dx) * DN_ROWB);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int tap = dz * 9 + dy * 3 + dx;
            bf16x8 B[NH];
#pragma unroll
            for (int h = 0; h < NH; ++h)
                B[h] = *reinterpret_cast<const bf16x8*>(bbase + (tap * NH + h) * 1024);
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int h = 0; h < NH; ++h)
                    acc[blk][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[blk + dy], B[h], acc[blk][h], 0, 0, 0);
        }
    }
}

// The 32 -> 3 layer with the output rows folded into the matrix columns:
// column 4 blk + c (c < 3; c = 3 is zero) of one MFMA holds output channel c
// of row block blk, so the halo row r (0..5) of a tap column (dz, dx) is one
// A fragment multiplied by one B fragment whose column (blk, c) carries the
// weight of tap (dz, r - blk, dx) when 0 <= r - blk <= 2 (else zero):
// 6 MFMAs per tap column instead of 12 (4 row blocks x 3 dy taps), 12 of the
// 16 columns useful instead of 3.  B fragment (zx, r) is rows
// 16 (6 zx + r) .. + 15 of the packed weights.
__device__ __forceinline__ void dn_mma3(const char* act, const char* wl, f32x4& acc) {
    const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int m = l & 15, q = l >> 4;
    const char* abase = act + (lz * DN_HY * DN_HX + m) * DN_ROWB + q * 16;
    const char* bbase = wl + dn_chunk(m, q);
#pragma unroll
    for (int zx = 0; zx < 9; ++zx) {
        const int dz = zx / 3, dx = zx % 3;
#pragma unroll
        for (int r = 0; r < DN_HY; ++r) {
            const bf16x8 A = *reinterpret_cast<const bf16x8*>(abase + ((dz * DN_HY + r) * DN_HX + dx) * DN_ROWB);
            const bf16x8 B = *reinterpret_cast<const bf16x8*>(bbase + (zx * DN_HY + r) * 1024);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc, 0, 0, 0);
        }
    }
}

}  // namespace pic
