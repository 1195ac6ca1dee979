// Device-side building blocks of the PIC cycle for gfx950 (CDNA4).
//
// Everything here is FP32 arithmetic with explicit fmaf (the library is
// compiled with -ffp-contract=off) so that each helper gives bit-identical
// results wherever it is inlined: the split kernels and the fused tiled
// kernel share these functions, which makes the two paths agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// Fixed-point scale of the current accumulator: 2^40 (resolution 9.1e-13,
// range +-8.4e6 in units of q w).  Sums of int64 are exact and independent
// of summation order; J is rounded to FP32 once, when it is read out.
#define PIC_FIX_SCALE 0x1p40f
#define PIC_FIX_INV 0x1p-40

// Kernel-side view of the grid.
struct Geom {
    int n[3];
    int nxy;
    int ncell;
    int window;    // 1: x is a moving-window circular buffer
    int origin;    // storage x index of window cell 0
    int kill_lo;   // window mode: particles in window cells < kill_lo are removed
    int kill_hi;   // window mode: particles in window cells > n[0] - 1 - kill_hi are removed
    int pml;       // transverse absorbing layer of pml cells at each y and z edge (0: y, z periodic);
                   // particles in its cells are removed
    float dt;
    float dtd[3];  // dt / d  (converts velocity to cells per step)
    float inv_d[3];
};

// Particle tiles: T cells per tile along each axis, nt tiles per axis (the
// last tile of an axis may be ragged), tcells = T[0]*T[1]*T[2] key slots per tile.
struct TileGeom {
    int T[3];
    int nt[3];
    int ntiles;
    int tcells;
};

// Stencil coefficients of the transverse smoothing S_d (perfect dispersion).
struct PDCoef {
    float alpha[3];  // centre of S_x, S_y, S_z
    float beta[3];   // beta_x, beta_y, beta_z
    float gam[3];    // gamma_yz, gamma_zx, gamma_xy
};

struct SpeciesDev {
    int* cell;
    float* off[3];
    float* u[3];
    float* w;
    int* id;
    float qmh;   // q dt / (2 m): the Boris half-step factor
    float mq;    // -q: sign/charge factor of the deposited current
};

struct PrevDev {
    int* cell;
    float* off[3];
};

// device error flags (bit set)
enum { ERR_CFL = 1, ERR_NONFINITE = 2, ERR_OVERFLOW = 4 };

// round(a b) as int64, round-half-even, for FP32 values a, b with |a b| < 2^51
// (a is a current contribution already scaled by 2^40, so the result is
// round(a b 2^40) on the 2^-40 grid).  The product of two FP32 values is exact
// in FP64, so one FMA onto M = 1.5 * 2^52, where doubles are spaced exactly 1
// apart, rounds the exact product once, half to even, to an integer; that
// integer is the difference of the bit patterns of the sum and of M (same
// exponent while |a b| < 2^51).  Two VALU instructions (the FMA and a 32-bit
// add on the high word, the low word of M being zero) instead of a float
// multiply and a general float -> int64 conversion.
__device__ __forceinline__ long long fix_mul(double a, double b) {
    const double M = 0x1.8p52;
    return __double_as_longlong(fma(a, b, M)) - __double_as_longlong(M);
}

__device__ __forceinline__ int wrapi(int i, int n) {
    // i in [-n, 2n)
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Cubic B-spline weights on nodes i-1, i, i+1, i+2 for a particle at i + d, d in [0, 1).
__device__ __forceinline__ void spline4(float d, float w[4]) {
    const float d2 = d * d;
    const float d3 = d2 * d;
    const float e = 1.0f - d;
    w[0] = e * e * e * (1.0f / 6.0f);
    w[1] = fmaf(0.5f, d3, (2.0f / 3.0f) - d2);
    w[2] = fmaf(0.5f, (d + d2) - d3, 1.0f / 6.0f);
    w[3] = d3 * (1.0f / 6.0f);
}

// Weights of the half-integer grid (nodes at j + 1/2): base offset relative to
// the particle's cell (-1 or -2) and the four weights.
__device__ __forceinline__ int spline4_half(float off, float w[4]) {
    if (off >= 0.5f) {
        spline4(off - 0.5f, w);
        return -1;
    }
    spline4(off + 0.5f, w);
    return -2;
}

// Tensor-product interpolation of one component: F[ix[a] + iy[b] + iz[c]]
// weighted by wx[a] wy[b] wz[c], summed x-innermost.
__device__ __forceinline__ float interp3(const float* __restrict__ F, const int ix[4], const int iy[4],
                                         const int iz[4], const float wx[4], const float wy[4],
                                         const float wz[4]) {
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        // the 16 values of one z-plane are loaded before any is used, so their
        // loads are in flight together
        float v[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float* row = F + (iz[c] + iy[b]);
#pragma unroll
            for (int a = 0; a < 4; ++a) v[b][a] = row[ix[a]];
        }
        float accy = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float ax = wx[0] * v[b][0];
            ax = fmaf(wx[1], v[b][1], ax);
            ax = fmaf(wx[2], v[b][2], ax);
            ax = fmaf(wx[3], v[b][3], ax);
            accy = fmaf(wy[b], ax, accy);
        }
        acc = fmaf(wz[c], accy, acc);
    }
    return acc;
}

// Per-particle interpolation stencil: weights and base offsets (relative to the
// particle's cell) of the integer and half-integer grids along each axis.
struct GatherStencil {
    float wi[3][4], wh[3][4];
    int hb[3];
};

__device__ __forceinline__ void gather_stencil(const float off[3], GatherStencil& s) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        spline4(off[d], s.wi[d]);
        s.hb[d] = spline4_half(off[d], s.wh[d]);
    }
}

// Relativistic Boris push (u = gamma v/c): u- = u + hE, t = hB/gamma-,
// s = 2t/(1+t^2), u' = u- + u- x t, u+ = u- + u' x s, u = u+ + hE.
__device__ __forceinline__ void boris(float u[3], const float E[3], const float B[3], float h) {
    const float um0 = fmaf(h, E[0], u[0]);
    const float um1 = fmaf(h, E[1], u[1]);
    const float um2 = fmaf(h, E[2], u[2]);
    const float gm = sqrtf(fmaf(um0, um0, fmaf(um1, um1, fmaf(um2, um2, 1.0f))));
    const float hg = h / gm;
    const float t0 = hg * B[0], t1 = hg * B[1], t2 = hg * B[2];
    const float tt = fmaf(t0, t0, fmaf(t1, t1, t2 * t2));
    const float f = 2.0f / (1.0f + tt);
    const float s0 = f * t0, s1 = f * t1, s2 = f * t2;
    const float up0 = um0 + (um1 * t2 - um2 * t1);
    const float up1 = um1 + (um2 * t0 - um0 * t2);
    const float up2 = um2 + (um0 * t1 - um1 * t0);
    const float uq0 = um0 + (up1 * s2 - up2 * s1);
    const float uq1 = um1 + (up2 * s0 - up0 * s2);
    const float uq2 = um2 + (up0 * s1 - up1 * s0);
    u[0] = fmaf(h, E[0], uq0);
    u[1] = fmaf(h, E[1], uq1);
    u[2] = fmaf(h, E[2], uq2);
}

// Move by `dc` cells along one axis with carry into the integer cell.
// |dc| < 1 is required (flagged by the caller otherwise).  Returns the carry
// (-1, 0, +1) and updates off in [0, 1).
__device__ __forceinline__ int move_carry(float& off, float dc) {
    float o = off + dc;
    int carry = 0;
    if (o >= 1.0f) {
        o -= 1.0f;   // exact for o in [1, 2)
        carry = 1;
    } else if (o < 0.0f) {
        o += 1.0f;
        carry = -1;
        if (o >= 1.0f) {   // |o| below half an ulp of 1: stay in the old cell at offset 0
            o = 0.0f;
            carry = 0;
        }
    }
    off = o;
    return carry;
}

// Differences w_t(a) - w_t(b), t = 0..3, of the cubic node weights, each
// factored as (a - b) q_t(a, b) so that small displacements keep their
// relative accuracy (no cancellation between two nearly equal weights).
__device__ __forceinline__ void dweight4(float a, float b, float D[4]) {
    const float dd = a - b;
    const float p = a + b;
    const float c = fmaf(a, a, fmaf(a, b, b * b));   // a^2 + ab + b^2
    D[0] = dd * (-(3.0f - 3.0f * p + c) * (1.0f / 6.0f));
    D[1] = dd * fmaf(0.5f, c, -p);
    D[2] = dd * (0.5f * ((1.0f + p) - c));
    D[3] = dd * (c * (1.0f / 6.0f));
}

// Esirkepov decomposition of one particle's motion along one axis.
// Old position: cell c0, offset d0; new: cell c0 + di, offset d1, di in {-1,0,1}.
// Union support: 5 nodes starting at c0 + base, base = min(0, di) - 1.
// S0[j]: old weights; dS[j] = S1[j] - S0[j].  Across a cell crossing each
// node's difference is split at the knot that the particle crosses
// (w_t(d1) - w_t(r1) + w_t'(r0) - w_t'(d0), r = 0 or 1), so every piece is a
// same-polynomial difference and keeps full relative accuracy.
struct Axis5 {
    float S0[5];
    float dS[5];
    int base;
    int len;   // 4 without a cell crossing, 5 with one
};

__device__ __forceinline__ void axis5(int di, float d0, float d1, Axis5& A) {
    A.base = (di < 0 ? di : 0) - 1;
    A.len = di == 0 ? 4 : 5;
    const float r1 = di == 0 ? d0 : (di > 0 ? 0.0f : 1.0f);
    const float r0 = di == 0 ? d0 : (di > 0 ? 1.0f : 0.0f);
    float W[4], Dn[4], Do[4];
    spline4(d0, W);
    dweight4(d1, r1, Dn);   // new-position piece, same polynomial as at r1
    dweight4(r0, d0, Do);   // old-position piece, same polynomial as at r0
    const bool so = di < 0;  // old weights sit one node further right in the union
    const bool sn = di > 0;  // new weights sit one node further right
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float wo = so ? (j >= 1 ? W[j - 1] : 0.0f) : (j <= 3 ? W[j] : 0.0f);
        const float dn = sn ? (j >= 1 ? Dn[j - 1] : 0.0f) : (j <= 3 ? Dn[j] : 0.0f);
        const float dO = so ? (j >= 1 ? Do[j - 1] : 0.0f) : (j <= 3 ? Do[j] : 0.0f);
        A.S0[j] = wo;
        A.dS[j] = dn + dO;
    }
}

}  // namespace pic
