// Per-particle steps of the PIC cycle shared by the split kernels and the
// fused tiled kernel (identical arithmetic in both).
#pragma once

#include "pic_device.h"

namespace pic {

__device__ __forceinline__ void decompose(const Geom& g, int cell, int c[3]) {
    const int cz = cell / g.nxy;
    const int r = cell - cz * g.nxy;
    const int cy = r / g.n[0];
    c[0] = r - cy * g.n[0];
    c[1] = cy;
    c[2] = cz;
}

// Moving window: particles outside window cells [kill_lo, n - 1 - kill_hi] are
// removed (their cubic shapes would reach across the window's ends).
__device__ __forceinline__ bool window_killed(const Geom& g, int cx) {
    if (!g.window) return false;
    int xw = cx - g.origin;
    if (xw < 0) xw += g.n[0];
    return xw < g.kill_lo || xw > g.n[0] - 1 - g.kill_hi;
}

// Removed at the start of a step: in a window kill zone, or in a transverse
// cell of the absorbing layer.
__device__ __forceinline__ bool particle_killed(const Geom& g, const int c[3]) {
    if (window_killed(g, c[0])) return true;
    if (g.pml == 0) return false;
    return c[1] < g.pml || c[1] >= g.n[1] - g.pml || c[2] < g.pml || c[2] >= g.n[2] - g.pml;
}

// Shift between two cell indices along a periodic axis, mapped to (-n/2, n/2].
__device__ __forceinline__ int unwrap_shift(int di, int n) {
    if (di > n / 2) di -= n;
    if (di < -(n / 2)) di += n;
    return di;
}

// Cubic gather of the six staggered components given the per-axis node index
// offsets (already multiplied by the axis stride) of the integer (ii) and
// half-integer (ih) grids.  E_x: x half, y, z integer; E_y: y half; E_z: z half;
// B_x: y, z half; B_y: x, z half; B_z: x, y half.
__device__ __forceinline__ void gather_fields(float* const E[3], float* const B[3], const int ii[3][4],
                                              const int ih[3][4], const GatherStencil& s, float Ep[3],
                                              float Bp[3]) {
    Ep[0] = interp3(E[0], ih[0], ii[1], ii[2], s.wh[0], s.wi[1], s.wi[2]);
    Ep[1] = interp3(E[1], ii[0], ih[1], ii[2], s.wi[0], s.wh[1], s.wi[2]);
    Ep[2] = interp3(E[2], ii[0], ii[1], ih[2], s.wi[0], s.wi[1], s.wh[2]);
    Bp[0] = interp3(B[0], ii[0], ih[1], ih[2], s.wi[0], s.wh[1], s.wh[2]);
    Bp[1] = interp3(B[1], ih[0], ii[1], ih[2], s.wh[0], s.wi[1], s.wh[2]);
    Bp[2] = interp3(B[2], ih[0], ih[1], ii[2], s.wh[0], s.wh[1], s.wi[2]);
}

// Boris push, then move by dt u / gamma with carry into the cell index
// (periodic wrap in storage coordinates).  Returns device error flags.
__device__ __forceinline__ int push_move(const Geom& g, float qmh, const float E[3], const float B[3], float u[3],
                                         float off[3], int c[3]) {
    boris(u, E, B, qmh);
    const float ig = 1.0f / sqrtf(fmaf(u[0], u[0], fmaf(u[1], u[1], fmaf(u[2], u[2], 1.0f))));
    int flags = 0;
    if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]))) {
        flags |= ERR_NONFINITE;
        u[0] = u[1] = u[2] = 0.0f;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float dc = (g.dtd[d] * u[d]) * ig;
        if (!(fabsf(dc) < 1.0f)) {   // a move of a cell or more breaks the deposit's support
            flags |= ERR_CFL;
            dc = dc > 0.0f ? 0.99f : -0.99f;
        }
        const int carry = move_carry(off[d], dc);
        c[d] = wrapi(c[d] + carry, g.n[d]);
    }
    return flags;
}

// True unless the particle kept its cell and offsets (then its current is zero).
__device__ __forceinline__ bool moved(const int c0[3], const int c1[3], const float o0[3], const float o1[3]) {
    return (c0[0] != c1[0]) | (c0[1] != c1[1]) | (c0[2] != c1[2]) | (o0[0] != o1[0]) | (o0[1] != o1[1]) |
           (o0[2] != o1[2]);
}

// Esirkepov current of one particle: for component x,
//   J_x[a][b][c] += (-q w) * P_x[a] * (M_y[b] M_z[c] + dS_y[b] dS_z[c] / 12)
// with P_x the running sum of dS_x along x and M = S0 + dS/2 (this product form
// equals dS_x (S0y S0z + dSy S0z/2 + S0y dSz/2 + dSy dSz/3) summed along x).
// Emit::add(comp, jx, jy, jz, k) receives each contribution as the int64
// k = round(2^40 (-q w) P Y), (jx, jy, jz) being union-node indices 0..4
// along x, y, z: the FP32 factor Q = 2^40 (-q w) Y is formed as
// fma((Q0 / 12) dS_y[b], dS_z[c], (Q0 M_y[b]) M_z[c]), Q0 = 2^40 (-q w), with
// the two scaled arrays of the first transverse axis computed once per
// component, and Q and P are multiplied exactly and rounded once.
// Callers skip particles that did not move (every contribution is zero).
//
// CELLREL: the indices passed to Emit::add are slots relative to the old
// cell instead of union nodes.  Along an axis transverse to the component,
// slots 0..3 are the nodes at cell - 1 .. cell + 2 whatever the crossing and
// slot 4 is the node a crossing adds (cell + 3 forward, cell - 2 backward);
// along the component's own axis slots 0..2 are cell - 1 .. cell + 1 and
// slot 3 is cell + 2 (forward) or cell - 2 (backward).  A backward crossing
// (union base -2) just rotates its arrays by one place, so every value goes
// to the same node as with union indices, bit for bit.
__device__ __forceinline__ void rotate_back5(bool back, float v[5]) {
    const float v0 = v[0];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = back ? v[j + 1] : v[j];
    v[4] = back ? v0 : v[4];
}

__device__ __forceinline__ void rotate_back4(bool back, float v[4]) {
    const float v0 = v[0];
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] = back ? v[j + 1] : v[j];
    v[3] = back ? v0 : v[3];
}

template <bool CELLREL = false, class Emit>
__device__ __forceinline__ void esirkepov(const Axis5 A[3], float qw, Emit& em) {
    const float qw40 = qw * PIC_FIX_SCALE;   // exact: a power-of-two scale
    const float qw12 = qw40 * (1.0f / 12.0f);
    float M[3][5], dS[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            M[d][j] = fmaf(0.5f, A[d].dS[j], A[d].S0[j]);
            dS[d][j] = A[d].dS[j];
        }
        if (CELLREL) {
            rotate_back5(A[d].base < -1, M[d]);
            rotate_back5(A[d].base < -1, dS[d]);
        }
    }
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const int t1 = comp == 0 ? 1 : (comp == 1 ? 2 : 0);
        const int t2 = comp == 0 ? 2 : (comp == 1 ? 0 : 1);
        float P[4];
        P[0] = A[comp].dS[0];
#pragma unroll
        for (int a = 1; a < 4; ++a) P[a] = P[a - 1] + A[comp].dS[a];
        if (CELLREL) rotate_back4(A[comp].base < -1, P);
        double Pd[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) Pd[a] = (double)P[a];
        const int la = A[comp].len - 1, lb = A[t1].len, lc = A[t2].len;
        float Mq[5], dSq[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            Mq[b] = qw40 * M[t1][b];
            dSq[b] = qw12 * dS[t1][b];
        }
#pragma unroll
        for (int cc = 0; cc < 5; ++cc) {
            if (cc >= lc) continue;
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                if (b >= lb) continue;
                const double qy = (double)fmaf(dSq[b], dS[t2][cc], Mq[b] * M[t2][cc]);
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    if (a >= la) continue;
                    const long long k = fix_mul(qy, Pd[a]);
                    if (comp == 0)
                        em.add(0, a, b, cc, k);
                    else if (comp == 1)
                        em.add(1, cc, a, b, k);
                    else
                        em.add(2, b, cc, a, k);
                }
            }
        }
    }
}

}  // namespace pic
