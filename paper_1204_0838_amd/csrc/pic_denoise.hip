// Learned current denoiser: the convolution layers of the network described
// in pic_dn_common.h and its output stage J' = B(J + sigma curl(y)).
// Inference runs layers 1, 2 (relu epilogues) and 3 (y), then the output
// stage; training reuses the same layer shapes for the gradient of the loss
// with respect to the activations (a transposed convolution is a
// convolution with the taps mirrored and the channel roles swapped) with a
// relu-mask epilogue, and the output stage with the loss.
#include <algorithm>

#include "pic_dn_common.h"

namespace pic {

// 32 output channels: EPI 0 = bf16 relu(acc + bias), 1 = bf16 acc where the
// mask activation is > 0.  The tile's 512 x 32 bf16 outputs are first placed
// in the LDS buffer ob (32 KB, rows swizzled like the inputs, so the 16 lanes
// of one cell and the 4 cells of one write hit different banks), then stored
// to HBM as whole 16-byte chunks of each cell.  The caller guarantees that no
// wavefront still reads ob; the function ends with ob free again only after
// the caller's next barrier.
template <int EPI>
__device__ __forceinline__ void dn_store32(const DnArgs& a, const int t0[3], const f32x4 acc[4][2], char* ob) {
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
                const int m = rq * 4 + j;
                float v;
                if (EPI == 0) {
                    v = fmaxf(acc[blk][h][j] + b, 0.0f);
                } else {
                    const int cell = dn_out_cell(a, t0, lz, blk, m);
                    v = cell >= 0 && (float)a.mask[(size_t)cell * 32 + co] > 0.0f ? acc[blk][h][j] : 0.0f;
                }
                const int lc = (lz * DN_TY + blk) * DN_TX + m;
                *reinterpret_cast<__bf16*>(ob + dn_chunk(lc, co >> 3) + (co & 7) * 2) = (__bf16)v;
            }
    }
    __syncthreads();
    constexpr int NCH = DN_TX * DN_TY * DN_TZ * 4;
#pragma unroll
    for (int k = 0; k < NCH / DN_THREADS; ++k) {
        const int g = threadIdx.x + k * DN_THREADS;
        const int lc = g >> 2, q = g & 3;
        const int m = lc % DN_TX, r = lc / DN_TX, blk = r % DN_TY, pz = r / DN_TY;
        const int cell = dn_out_cell(a, t0, pz, blk, m);
        if (cell >= 0)
            reinterpret_cast<uint4*>(a.act_out)[(size_t)cell * 4 + q] = *reinterpret_cast<const uint4*>(ob + dn_chunk(lc, q));
    }
}

// 4-channel input (3 used), 32 output channels.  K = tap * 4 + channel
// (channel 3 and taps 27..31 zero), 4 K-steps of 32; lane chunk q of step s
// covers taps 8s + 2q and 8s + 2q + 1.  IN 0: the current J_d / s_d (FP32,
// rounded to bf16 here); IN 1: a bf16 [cell][4] array.
template <int IN, int EPI>
__global__ void __launch_bounds__(DN_THREADS) k_dn_c4(DnArgs a) {
    __shared__ __attribute__((aligned(16))) char lds[DN_HCELLS * 8 + 32 * 256 + DN_TX * DN_TY * DN_TZ * 64];
    char* xin = lds;                       // [halo cell][4] bf16
    char* wl = lds + DN_HCELLS * 8;        // [co][128] bf16, 256 B rows
    char* ob = wl + 32 * 256;              // output tile (dn_store32)
    int t0[3];
    dn_tile(t0);
    {
        const uint4* src = reinterpret_cast<const uint4*>(a.w);
        for (int g = threadIdx.x; g < 32 * 16; g += DN_THREADS) reinterpret_cast<uint4*>(wl)[g] = src[g];
    }
    {
        // every global load of the thread first, then the LDS stores
        constexpr int PER = (DN_HCELLS + DN_THREADS - 1) / DN_THREADS;
        bf16x4 v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int c = threadIdx.x + k * DN_THREADS;
            const int hx = c % DN_HX, r = c / DN_HX, hy = r % DN_HY, hz = r / DN_HY;
            v[k] = bf16x4{(__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
            if (c < DN_HCELLS && hx < DN_TX + 2) {
                const int s = dn_halo_src(a, t0, hx, hy, hz);
                if (s >= 0) {
                    if (IN == 0) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) v[k][d] = (__bf16)(a.J[d][s] * a.inv_scale[d]);
                    } else {
                        v[k] = reinterpret_cast<const bf16x4*>(a.c4_in)[s];
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int c = threadIdx.x + k * DN_THREADS;
            if (c < DN_HCELLS) *reinterpret_cast<bf16x4*>(xin + c * 8) = v[k];
        }
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
    dn_store32<EPI>(a, t0, acc, ob);
}

// Layers with a 32-channel input: 32 -> 32 channels (KIND 0: relu(acc + b),
// 1: mask epilogue) or 32 -> 3 (KIND 2, the row blocks folded into the
// matrix columns, dn_mma3: y = acc + b as FP32 components into a.Jout).  Persistent: one workgroup per compute unit stages
// the weights once and walks the tiles t = blockIdx.x, + gridDim.x, ...; the
// next tile's input halo is loaded into registers while the current tile's
// matrix work runs.
template <int KIND>
__global__ void __launch_bounds__(DN_THREADS) k_dn_conv32(DnArgs a) {
    constexpr int NH = KIND == 2 ? 1 : 2;
    extern __shared__ __attribute__((aligned(16))) char dlds[];
    char* act = dlds;
    char* wl = dlds + DN_ACT_LDS;
    int ntx, nty;
    const int ntiles = dn_ntiles(a.n, &ntx, &nty);
    dn_stage_weights<KIND == 2 ? 9 * DN_HY * 16 : 27 * 16 * NH>(a.w, wl);
    // XCD-aware walk (workgroups go round-robin over the 8 XCDs): the
    // workgroups of one XCD share a contiguous range of tiles and walk it
    // together, so the halos they share stay in that XCD's L2
    int tile, stride, end;
    if (gridDim.x % 8 == 0) {
        const int per = (ntiles + 7) / 8, k = blockIdx.x % 8;
        tile = k * per + blockIdx.x / 8;
        stride = gridDim.x / 8;
        end = min(ntiles, (k + 1) * per);
    } else {
        tile = blockIdx.x;
        stride = gridDim.x;
        end = ntiles;
    }
    int t0[3];
    int hc[DN_ACT_PER];
    dn_halo_coords(hc);
    const DnBox box = dn_box(a);
    uint4 v[DN_ACT_PER];
    if (tile < end) {
        dn_tile_of(tile, ntx, nty, t0);
        dn_load_act(a, box, t0, hc, v);
    }
    while (tile < end) {
        __syncthreads();   // the previous tile's LDS reads are done (first pass: nothing)
        dn_store_act(v, act);
        __syncthreads();   // halo (and, first pass, weights) staged
        const int cur[3] = {t0[0], t0[1], t0[2]};
        const int next = tile + stride;
        if (next < end) {
            dn_tile_of(next, ntx, nty, t0);
            dn_load_act(a, box, t0, hc, v);
        }
        if constexpr (KIND == 2) {
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            dn_mma3(act, wl, acc);
            const int l = threadIdx.x & 63, lz = threadIdx.x >> 6;
            const int col = l & 15, rq = l >> 4;
            const int blk = col >> 2, co = col & 3;
            if (co < 3) {
                // pick the component's pointer among the three (indexing the
                // argument array with a lane value would re-read it from memory)
                float* out = co == 0 ? a.Jout[0] : (co == 1 ? a.Jout[1] : a.Jout[2]);
                const float b = a.bias[co];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int cell = dn_out_cell(a, cur, lz, blk, rq * 4 + j);
                    if (cell >= 0) out[cell] = acc[j] + b;
                }
            }
        } else {
            f32x4 acc[4][NH];
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int h = 0; h < NH; ++h) acc[blk][h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            dn_mma32<NH>(act, wl, acc);
            __syncthreads();   // every wavefront is done reading the halo: reuse it for the output tile
            dn_store32<KIND>(a, cur, acc, act);
        }
        tile = next;
    }
}

// Window/box coordinates of cell index i (x fastest), its storage index,
// and the storage indices of neighbours (-1 = zero).
struct DnCell {
    int w[3];
    int s;
};

__device__ __forceinline__ int dn_nb(const DnCombine& c, const DnCell& k, int dx, int dy, int dz) {
    const int x = dn_axis(k.w[0] + dx, c.n[0], c.bc[0], c.origin);
    const int y = dn_axis(k.w[1] + dy, c.n[1], c.bc[1], 0);
    const int z = dn_axis(k.w[2] + dz, c.n[2], c.bc[2], 0);
    if (x < 0 || y < 0 || z < 0) return -1;
    return x + c.n[0] * (y + c.n[1] * z);
}

__device__ __forceinline__ bool dn_cell(const DnCombine& c, int i, DnCell& k) {
    if (i >= c.n[0] * c.n[1] * c.n[2]) return false;
    k.w[0] = i % c.n[0];
    const int r = i / c.n[0];
    k.w[1] = r % c.n[1];
    k.w[2] = r / c.n[1];
    k.s = dn_nb(c, k, 0, 0, 0);
    return true;
}

__device__ __forceinline__ float dn_at(const float* __restrict__ F, int s) { return s >= 0 ? F[s] : 0.0f; }

// dst = src + sigma curl(y), curl(y)_a = (y_{a+2} - y_{a+2}[-e_{a+1}]) / d_{a+1} - (y_{a+1} - y_{a+1}[-e_{a+2}]) / d_{a+2}.
__global__ void __launch_bounds__(256) k_dn_curl_add(DnCombine c) {
    DnCell k;
    if (!dn_cell(c, blockIdx.x * blockDim.x + threadIdx.x, k)) return;
    const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const int t1 = (comp + 1) % 3, t2 = (comp + 2) % 3;
        const int m1 = dn_nb(c, k, -off[t1][0], -off[t1][1], -off[t1][2]);
        const int m2 = dn_nb(c, k, -off[t2][0], -off[t2][1], -off[t2][2]);
        const float cu = (c.y[t2][k.s] - dn_at(c.y[t2], m1)) * c.inv_d[t1] -
                         (c.y[t1][k.s] - dn_at(c.y[t1], m2)) * c.inv_d[t2];
        c.dst[comp][k.s] = fmaf(c.sigma, cu, c.src[comp][k.s]);
    }
}

// Binomial filter of src (27-point product stencil, x innermost).
template <bool LOSS>
__device__ __forceinline__ void dn_binomial_cell(const DnCombine& c, const DnCell& k, double& part) {
    const float w[3] = {0.25f, 0.5f, 0.25f};
    int nb[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) nb[q] = dn_nb(c, k, q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1);
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        float acc = 0.0f;
#pragma unroll
        for (int zc = 0; zc < 3; ++zc) {
            float ay = 0.0f;
#pragma unroll
            for (int yb = 0; yb < 3; ++yb) {
                float ax = 0.0f;
#pragma unroll
                for (int xa = 0; xa < 3; ++xa) ax = fmaf(w[xa], dn_at(c.src[comp], nb[(zc * 3 + yb) * 3 + xa]), ax);
                ay = fmaf(w[yb], ax, ay);
            }
            acc = fmaf(w[zc], ay, acc);
        }
        if (LOSS) {
            const float e = (acc - c.T[comp][k.s]) * c.inv_scale[comp];
            part += (double)e * (double)e;
            c.dst[comp][k.s] = c.grad_scale * e * c.inv_scale[comp];
        } else {
            c.dst[comp][k.s] = acc;
        }
    }
}

template <bool LOSS>
__global__ void __launch_bounds__(256) k_dn_binomial(DnCombine c) {
    DnCell k;
    const bool ok = dn_cell(c, blockIdx.x * blockDim.x + threadIdx.x, k);
    double part = 0.0;
    if (ok) dn_binomial_cell<LOSS>(c, k, part);
    if (LOSS) {   // every lane takes part in the wavefront reduction
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(c.loss, part * (0.5 * (double)c.grad_scale));
    }
}

// dy = sigma curl^T(src): dy_a = sigma [(src_{a+2}(p + e_{a+1}) - src_{a+2}(p)) / d_{a+1}
//                                       - (src_{a+1}(p + e_{a+2}) - src_{a+1}(p)) / d_{a+2}]
// (the forward-difference curl), as bf16 [cell][4] with channel 3 zero.
__global__ void __launch_bounds__(256) k_dn_curl_adjoint(DnCombine c) {
    DnCell k;
    if (!dn_cell(c, blockIdx.x * blockDim.x + threadIdx.x, k)) return;
    const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    bf16x4 out;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        const int p1 = dn_nb(c, k, off[a1][0], off[a1][1], off[a1][2]);
        const int p2 = dn_nb(c, k, off[a2][0], off[a2][1], off[a2][2]);
        const float v = (dn_at(c.src[a2], p1) - c.src[a2][k.s]) * c.inv_d[a1] -
                        (dn_at(c.src[a1], p2) - c.src[a1][k.s]) * c.inv_d[a2];
        out[a] = (__bf16)(c.sigma * v);
    }
    out[3] = (__bf16)0.0f;
    reinterpret_cast<bf16x4*>(c.dy)[k.s] = out;
}

// Inference output stage fused in one pass over tiles of 32 x 8 x 4 cells:
// J' = B(t), t = J + sigma curl(y), with t computed in LDS on the tile plus a
// 1-cell halo (zero outside the box) from y staged with a further cell below
// (the backward differences).  Same arithmetic, in the same order, as
// k_dn_curl_add followed by k_dn_binomial<false>.
constexpr int DO_TX = 32, DO_TY = 8, DO_TZ = 4, DO_THREADS = DO_TX * DO_TY * DO_TZ;
constexpr int DO_YX = DO_TX + 3, DO_YY = DO_TY + 3, DO_YZ = DO_TZ + 3;   // y: cells -2 .. T
constexpr int DO_SX = DO_TX + 2, DO_SY = DO_TY + 2, DO_SZ = DO_TZ + 2;   // t: cells -1 .. T

__device__ __forceinline__ int do_src(const DnCombine& c, int x, int y, int z) {
    const int sx = dn_axis(x, c.n[0], c.bc[0], c.origin);
    const int sy = dn_axis(y, c.n[1], c.bc[1], 0);
    const int sz = dn_axis(z, c.n[2], c.bc[2], 0);
    if (sx < 0 || sy < 0 || sz < 0) return -1;
    return sx + c.n[0] * (sy + c.n[1] * sz);
}

__global__ void __launch_bounds__(DO_THREADS) k_dn_output(DnCombine c) {
    __shared__ float ys[3][DO_YZ * DO_YY * DO_YX];
    __shared__ float ts[3][DO_SZ * DO_SY * DO_SX];
    const int t0[3] = {(int)blockIdx.x * DO_TX, (int)blockIdx.y * DO_TY, (int)blockIdx.z * DO_TZ};
    // Every global load of a thread is issued before the first of them is
    // used (the y halo, then the current at the t cells, the latter in flight
    // while the y halo is stored), so each staging pass waits for one memory
    // latency rather than one per cell.
    constexpr int NY = DO_YZ * DO_YY * DO_YX, PY = (NY + DO_THREADS - 1) / DO_THREADS;
    constexpr int NT = DO_SZ * DO_SY * DO_SX, PT = (NT + DO_THREADS - 1) / DO_THREADS;
    float yv[PY][3];
#pragma unroll
    for (int q = 0; q < PY; ++q) {
        const int i = (int)threadIdx.x + q * DO_THREADS;
        const int hx = i % DO_YX, r = i / DO_YX, hy = r % DO_YY, hz = r / DO_YY;
        const int s = i < NY ? do_src(c, t0[0] - 2 + hx, t0[1] - 2 + hy, t0[2] - 2 + hz) : -1;
#pragma unroll
        for (int d = 0; d < 3; ++d) yv[q][d] = dn_at(c.y[d], s);
    }
    int ts_src[PT];
    float sv[PT][3];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const int i = (int)threadIdx.x + q * DO_THREADS;
        const int hx = i % DO_SX, r = i / DO_SX, hy = r % DO_SY, hz = r / DO_SY;
        ts_src[q] = i < NT ? do_src(c, t0[0] - 1 + hx, t0[1] - 1 + hy, t0[2] - 1 + hz) : -1;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) sv[q][comp] = dn_at(c.src[comp], ts_src[q]);
    }
#pragma unroll
    for (int q = 0; q < PY; ++q) {
        const int i = (int)threadIdx.x + q * DO_THREADS;
        if (i < NY)
#pragma unroll
            for (int d = 0; d < 3; ++d) ys[d][i] = yv[q][d];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const int i = (int)threadIdx.x + q * DO_THREADS;
        if (i >= NT) continue;
        const int hx = i % DO_SX, r = i / DO_SX, hy = r % DO_SY, hz = r / DO_SY;
        const int s = ts_src[q];
        const int yc = ((hz + 1) * DO_YY + (hy + 1)) * DO_YX + (hx + 1);   // the same cell in ys
        const int ym[3] = {yc - 1, yc - DO_YX, yc - DO_YX * DO_YY};          // one cell lower along x, y, z
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
            const int t1 = (comp + 1) % 3, t2 = (comp + 2) % 3;
            float v = 0.0f;
            if (s >= 0) {
                const float cu = (ys[t2][yc] - ys[t2][ym[t1]]) * c.inv_d[t1] - (ys[t1][yc] - ys[t1][ym[t2]]) * c.inv_d[t2];
                v = fmaf(c.sigma, cu, sv[q][comp]);
            }
            ts[comp][i] = v;
        }
    }
    __syncthreads();
    const int lx = threadIdx.x % DO_TX, ly = (threadIdx.x / DO_TX) % DO_TY, lz = threadIdx.x / (DO_TX * DO_TY);
    const int x = t0[0] + lx, y = t0[1] + ly, z = t0[2] + lz;
    if (x >= c.n[0] || y >= c.n[1] || z >= c.n[2]) return;
    const int s = do_src(c, x, y, z);
    const float w[3] = {0.25f, 0.5f, 0.25f};
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        float acc = 0.0f;
#pragma unroll
        for (int zc = 0; zc < 3; ++zc) {
            float ay = 0.0f;
#pragma unroll
            for (int yb = 0; yb < 3; ++yb) {
                float ax = 0.0f;
                const int row = ((lz + zc) * DO_SY + (ly + yb)) * DO_SX + lx;
#pragma unroll
                for (int xa = 0; xa < 3; ++xa) ax = fmaf(w[xa], ts[comp][row + xa], ax);
                ay = fmaf(w[yb], ax, ay);
            }
            acc = fmaf(w[zc], ay, acc);
        }
        c.dst[comp][s] = acc;
    }
}

hipError_t launch_dn_output(const DnCombine& c, hipStream_t st) {
    const dim3 g((c.n[0] + DO_TX - 1) / DO_TX, (c.n[1] + DO_TY - 1) / DO_TY, (c.n[2] + DO_TZ - 1) / DO_TZ);
    hipLaunchKernelGGL(k_dn_output, g, dim3(DO_THREADS), 0, st, c);
    return hipGetLastError();
}

static dim3 dn_cells_grid(const DnCombine& c) { return dim3((c.n[0] * c.n[1] * c.n[2] + 255) / 256); }

hipError_t launch_dn_curl_add(const DnCombine& c, hipStream_t st) {
    hipLaunchKernelGGL(k_dn_curl_add, dn_cells_grid(c), dim3(256), 0, st, c);
    return hipGetLastError();
}

hipError_t launch_dn_binomial(const DnCombine& c, bool loss, hipStream_t st) {
    if (loss)
        hipLaunchKernelGGL(k_dn_binomial<true>, dn_cells_grid(c), dim3(256), 0, st, c);
    else
        hipLaunchKernelGGL(k_dn_binomial<false>, dn_cells_grid(c), dim3(256), 0, st, c);
    return hipGetLastError();
}

hipError_t launch_dn_curl_adjoint(const DnCombine& c, hipStream_t st) {
    hipLaunchKernelGGL(k_dn_curl_adjoint, dn_cells_grid(c), dim3(256), 0, st, c);
    return hipGetLastError();
}

static size_t dn_lds(int weight_rows) { return (size_t)DN_ACT_LDS + (size_t)weight_rows * 64; }

template <class K>
static hipError_t dn_launch(K kern, size_t lds, const DnArgs& a, hipStream_t st) {
    if (lds > 0) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dn_grid(a.n), dim3(DN_THREADS), lds, st, a);
    return hipGetLastError();
}

// Persistent layers: one workgroup per compute unit (their LDS allows one),
// never more than there are tiles.
template <class K>
static hipError_t dn_launch_persistent(K kern, size_t lds, const DnArgs& a, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, ncu = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const dim3 g = dn_grid(a.n);
    const long long ntiles = (long long)g.x * g.y * g.z;
    long long nb = std::max(1LL, std::min<long long>(ntiles, ncu > 0 ? ncu : 256));
    if (nb >= 8) nb -= nb % 8;   // a multiple of the 8 XCDs: the XCD-aware walk
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(DN_THREADS), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dn_layer(int kind, const DnArgs& a, hipStream_t st) {
    switch (kind) {
        case DN_L1_J_ACT: return dn_launch(k_dn_c4<0, 0>, 0, a, st);
        case DN_L1_C4_MASK: return dn_launch(k_dn_c4<1, 1>, 0, a, st);
        case DN_L2_ACT: return dn_launch_persistent(k_dn_conv32<0>, dn_lds(27 * 32), a, st);
        case DN_L2_MASK: return dn_launch_persistent(k_dn_conv32<1>, dn_lds(27 * 32), a, st);
        case DN_L3_Y: return dn_launch_persistent(k_dn_conv32<2>, dn_lds(9 * DN_HY * 16), a, st);
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
    // y (3 FP32 components) reuses the first activation buffer
    const size_t N = (size_t)g.ncell;
    float* y = reinterpret_cast<float*>(h1);
    a.act_in = h2;
    a.act_out = nullptr;
    a.w = w.w3;
    a.bias = w.b3;
    for (int d = 0; d < 3; ++d) a.Jout[d] = y + d * N;
    e = launch_dn_layer(DN_L3_Y, a, st);
    if (e != hipSuccess) return e;
    // J' = B(J + sigma curl(y)) in one pass (Jout must not alias Jin: tiles
    // read their neighbours' J)
    DnCombine c{};
    for (int d = 0; d < 3; ++d) {
        c.n[d] = g.n[d];
        c.bc[d] = bc[d];
        c.src[d] = Jin[d];
        c.y[d] = y + d * N;
        c.dst[d] = Jout[d];
        c.inv_d[d] = w.inv_d[d];
    }
    c.origin = a.origin;
    c.sigma = w.sigma;
    return launch_dn_output(c, st);
}

}  // namespace pic
