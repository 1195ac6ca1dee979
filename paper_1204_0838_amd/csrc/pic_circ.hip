// Quasi-cylindrical particle-in-cell step with the two lowest azimuthal
// modes (Section 1: fields and currents decomposed into poloidal modes on a
// radial grid while the macroparticles keep their full 3D Cartesian motion;
// Section 3.1 runs with m = 0, 1), on gfx950.
//
// Particle work (gather of both modes at each component's staggered
// position, relativistic Boris push, Cartesian move, charge-conserving
// deposit of J_z, J_r and J_th per mode) is one device routine used by the
// fused tiled kernel (fields of a tile and its halo staged in LDS, the
// tile's current summed in LDS as int64 fixed point and added to the global
// accumulator once), by the split gather/push and deposit kernels, and by
// the rest pass (particles beyond their tile's guard and those injected since
// the last sort): all paths give the same bits.
//
// The discretisation follows the readings written out in full beside the
// FP64 reference: linear shapes in z; a density-conserving linear shape in r
// (node K+1 of a particle at (K + s) dr gets s + s(1 - s)/(2(2K + 1)), so a
// uniform 3D density deposits n V_j on every node, the axis node included);
// half-node components interpolated linearly against a ghost at -dr/2 with
// the mode's axis parity; Esirkepov's decomposition of the change of
// a_i b_j kappa exp(i m th) into W_z, W_r, W_th.
#include "pic_circ_internal.h"

namespace pic {

namespace {

// ------------------------------------------------------------------ field access

// Field and accumulator access through a per-particle handle: at(bz, br)
// fixes the particle's base node once, and get / add address the node
// (bz + a, br + b) relative to it (a, b small constants), so the local
// accessors need one offset per base instead of one wrap per node.

// Global-memory reads: node (iz storage, jr); zero at or beyond the wall and
// below the axis.
struct GField {
    const CircGeom* g;
    const CircFields* F;
    struct H {
        int bz, br;
    };
    __device__ __forceinline__ H at(int bz, int br) const { return H{bz, br}; }
    __device__ __forceinline__ float get(const H& h, int f, int c, int ch, int a, int b) const {
        const int jr = h.br + b;
        if (jr < 0 || jr >= g->nr) return 0.0f;
        int iz = h.bz + a;
        iz = iz < 0 ? iz + g->nz : (iz >= g->nz ? iz - g->nz : iz);
        return F->F[f][c][ch][iz + g->nz * jr];
    }
};

// LDS reads: the tile's staged planes [18][SR][SZ], origin (fz0, fr0); rows
// below the axis and beyond the wall are staged as zero.
struct LField {
    const float* s;
    int fz0, fr0, nz;
    int SZ, SR;
    struct H {
        int o;
    };
    __device__ __forceinline__ H at(int bz, int br) const {
        int dz = bz - fz0;
        if (dz < 0) dz += nz;
        else if (dz >= nz) dz -= nz;
        return H{(br - fr0) * SZ + dz};
    }
    __device__ __forceinline__ float get(const H& h, int f, int c, int ch, int a, int b) const {
        return s[((f * 3 + c) * 3 + ch) * (SZ * SR) + h.o + b * SZ + a];
    }
};

// Global-memory int64 accumulator: [9][ncell].
struct GAcc {
    unsigned long long* a;
    int nz, ncell;
    struct H {
        int bz, br;
    };
    __device__ __forceinline__ H at(int bz, int br) const { return H{bz, br}; }
    __device__ __forceinline__ void add(const H& h, int ch, int da, int db, long long v) const {
        const int jr = h.br + db;
        if (v == 0 || jr < 0 || jr >= ncell / nz) return;
        int iz = h.bz + da;
        iz = iz < 0 ? iz + nz : (iz >= nz ? iz - nz : iz);
        atomicAdd(a + (size_t)ch * ncell + iz + nz * jr, (unsigned long long)v);
    }
};

// LDS int64 accumulator: [9][AR][AZ], origin (az0, ar0) (a zero adds nothing).
struct LAcc {
    unsigned long long* a;
    int az0, ar0, nz, AZ, AR;
    struct H {
        int o;
    };
    __device__ __forceinline__ H at(int bz, int br) const {
        int dz = bz - az0;
        if (dz < 0) dz += nz;
        else if (dz >= nz) dz -= nz;
        return H{(br - ar0) * AZ + dz};
    }
    __device__ __forceinline__ void add(const H& h, int ch, int da, int db, long long v) const {
        atomicAdd(a + ch * AR * AZ + h.o + db * AZ + da, (unsigned long long)v);
    }
};

// ------------------------------------------------------------------ gather

// Linear weights in z of the integer (sh = 0) or half (sh = 1) nodes: base node, weights.
__device__ __forceinline__ int zw(int iz, float oz, bool half, float w[2]) {
    if (!half) {
        w[0] = 1.0f - oz;
        w[1] = oz;
        return iz;
    }
    if (oz >= 0.5f) {
        const float t = oz - 0.5f;
        w[0] = 1.0f - t;
        w[1] = t;
        return iz;
    }
    const float t = oz + 0.5f;
    w[0] = 1.0f - t;
    w[1] = t;
    return iz - 1;
}

// One mode channel of one component at the particle from the 2 x 2 nodes at
// handle h.  wr: the radial weights with the axis ghost already folded in
// (see circ_gather).
template <class FA>
__device__ __forceinline__ float interp(const FA& fa, const typename FA::H& h, int f, int c, int ch,
                                        const float wz[2], const float wr[2]) {
    float acc = 0.0f;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) acc = fmaf(wz[a] * wr[b], fa.get(h, f, c, ch, a, b), acc);
    return acc;
}

// E, B (Cartesian x, y, z) at a particle in cell iz with z offset oz, at (x, y).
template <class FA>
__device__ __forceinline__ void circ_gather(const CircGeom& g, const FA& fa, int iz, float oz, float x, float y,
                                            float E[3], float B[3]) {
    float r, s;
    int K;
    circ_rcell(x, y, g.inv_dr, r, K, s);
    const float f1 = circ_fr(K, s);
    const float wri[2] = {1.0f - f1, f1};
    const float th = r * g.inv_dr - 0.5f;
    const int Kh = (int)floorf(th);
    const float sh = th - (float)Kh;
    // half-r nodes below dr/2 (Kh = -1): the ghost at -dr/2 is the node at dr/2
    // times the channel's axis parity, so its weight moves onto that node
    const bool ghost = Kh < 0;
    const float wrh[2] = {ghost ? 0.0f : 1.0f - sh, sh};
    const float wrg_even[2] = {0.0f, ghost ? sh + (1.0f - sh) : sh};     // parity +1
    const float wrg_odd[2] = {0.0f, ghost ? sh - (1.0f - sh) : sh};      // parity -1
    float wzi[2], wzh[2];
    const int bzi = zw(iz, oz, false, wzi);
    const int bzh = zw(iz, oz, true, wzh);
    const typename FA::H h_ii = fa.at(bzi, K), h_hi = fa.at(bzh, K), h_ih = fa.at(bzi, Kh), h_hh = fa.at(bzh, Kh);
    const float inv_r = r > 0.0f ? 1.0f / r : 0.0f;
    const float ct = r > 0.0f ? x * inv_r : 1.0f;
    const float st = r > 0.0f ? y * inv_r : 0.0f;
    float comp[2][3];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // staggering: E_z (half z, int r), E_r (int z, half r), E_th (int, int);
            //             B_z (int z, half r), B_r (half z, int r), B_th (half, half)
            const bool zhalf = f == 0 ? c == 0 : c != 0;
            const bool rhalf = f == 0 ? c == 1 : c != 1;
            // axis parity of the half-r ghost: r, th components odd for m 0 and even
            // for m 1; the z component the other way round
            const bool z_comp = c == 0;
            const float* wz = zhalf ? wzh : wzi;
            const typename FA::H& h = zhalf ? (rhalf ? h_hh : h_hi) : (rhalf ? h_ih : h_ii);
            const float* w0 = rhalf ? (ghost ? (z_comp ? wrg_even : wrg_odd) : wrh) : wri;   // m 0 channel
            const float* w1 = rhalf ? (ghost ? (z_comp ? wrg_odd : wrg_even) : wrh) : wri;   // m 1 channels
            const float v0 = interp(fa, h, f, c, 0, wz, w0);
            const float v1 = interp(fa, h, f, c, 1, wz, w1);
            const float v2 = interp(fa, h, f, c, 2, wz, w1);
            comp[f][c] = v0 + fmaf(v1, ct, v2 * st);
        }
    }
    E[0] = comp[0][1] * ct - comp[0][2] * st;
    E[1] = comp[0][1] * st + comp[0][2] * ct;
    E[2] = comp[0][0];
    B[0] = comp[1][1] * ct - comp[1][2] * st;
    B[1] = comp[1][1] * st + comp[1][2] * ct;
    B[2] = comp[1][0];
}

// ------------------------------------------------------------------ push

struct CircParticle {
    int iz, jr;        // cell (storage z, r)
    float oz, x, y;    // z offset, transverse position
    float u[3];
    float w;
};

// Gather + Boris + move.  Returns an error flag (ERR_NONFINITE, ERR_CFL: a
// move of a cell or more along z) and leaves the particle unmoved then, else 0.
template <class FA>
__device__ __forceinline__ int circ_push(const CircGeom& g, const FA& fa, float qmh, const CircParticle& p0,
                                         CircParticle& p1) {
    float E[3], B[3];
    circ_gather(g, fa, p0.iz, p0.oz, p0.x, p0.y, E, B);
    p1 = p0;
    boris(p1.u, E, B, qmh);
    const float gi = 1.0f / sqrtf(fmaf(p1.u[0], p1.u[0], fmaf(p1.u[1], p1.u[1], fmaf(p1.u[2], p1.u[2], 1.0f))));
    if (!isfinite(p1.u[0]) || !isfinite(p1.u[1]) || !isfinite(p1.u[2])) {
        p1 = p0;
        return ERR_NONFINITE;
    }
    const float dcz = g.dtdz * (p1.u[2] * gi);
    if (!(fabsf(dcz) < 1.0f)) {
        p1 = p0;
        return ERR_CFL;
    }
    p1.x = fmaf(g.dt, p1.u[0] * gi, p0.x);
    p1.y = fmaf(g.dt, p1.u[1] * gi, p0.y);
    p1.iz = p0.iz + move_carry(p1.oz, dcz);
    if (p1.iz < 0) p1.iz += g.nz;
    else if (p1.iz >= g.nz) p1.iz -= g.nz;
    float r, s;
    circ_rcell(p1.x, p1.y, g.inv_dr, r, p1.jr, s);
    return 0;
}

// ------------------------------------------------------------------ deposit

// Charge-conserving deposit of the move p0 -> p1 (u of p1 is u^{n+1/2}).
// c = kappa exp(i m th): m 0 -> 1, m 1 -> 2 (cos th + i sin th).
template <class AC>
__device__ __forceinline__ void circ_deposit(const CircGeom& g, const AC& acc, float q, const CircParticle& p0,
                                             const CircParticle& p1) {
    // A particle that kept its cell and position and has no transverse momentum
    // contributes exactly zero to every mode (the charge-conserving parts are
    // products of the position changes, the direct m = 0 azimuthal part is
    // proportional to x u_y - y u_x): skip it (a cold plasma ahead of the pulse).
    if (p1.iz == p0.iz && p1.oz == p0.oz && p1.x == p0.x && p1.y == p0.y && p1.u[0] == 0.0f && p1.u[1] == 0.0f)
        return;
    float r0, s0, r1, s1;
    int K0, K1;
    circ_rcell(p0.x, p0.y, g.inv_dr, r0, K0, s0);
    circ_rcell(p1.x, p1.y, g.inv_dr, r1, K1, s1);
    int carry = p1.iz - p0.iz;
    if (carry > 1) carry -= g.nz;
    else if (carry < -1) carry += g.nz;
    const int bz = p0.iz + (carry < 0 ? -1 : 0);      // union support base (storage, may be -1)
    const int br = K0 < K1 ? K0 : K1;
    // z weights on nodes bz..bz+2; differences summing to zero exactly
    float a0[3] = {0.0f, 0.0f, 0.0f}, a1[3] = {0.0f, 0.0f, 0.0f};
    const int o0 = p0.iz + (carry < 0 ? 1 : 0) - p0.iz;   // node offset of p0's base in the union
    const int o1 = o0 + carry;
    a0[o0] = 1.0f - p0.oz;
    a0[o0 + 1] = p0.oz;
    a1[o1] += 1.0f - p1.oz;
    a1[o1 + 1] += p1.oz;
    float da[3];
    da[1] = a1[1] - a0[1];
    da[2] = a1[2] - a0[2];
    da[0] = -(da[1] + da[2]);
    const float f0 = circ_fr(K0, s0), f1 = circ_fr(K1, s1);
    float b0[3] = {0.0f, 0.0f, 0.0f}, b1[3] = {0.0f, 0.0f, 0.0f};
    b0[K0 - br] = 1.0f - f0;
    b0[K0 - br + 1] = f0;
    b1[K1 - br] += 1.0f - f1;
    b1[K1 - br + 1] += f1;
    float db[3];
    db[1] = b1[1] - b0[1];
    db[2] = b1[2] - b0[2];
    db[0] = -(db[1] + db[2]);
    // phases kappa exp(i th)
    const float k0 = r0 > 0.0f ? 2.0f / r0 : 0.0f, k1 = r1 > 0.0f ? 2.0f / r1 : 0.0f;
    const float c0r = r0 > 0.0f ? p0.x * k0 : 2.0f, c0i = r0 > 0.0f ? p0.y * k0 : 0.0f;
    const float c1r = r1 > 0.0f ? p1.x * k1 : 2.0f, c1i = r1 > 0.0f ? p1.y * k1 : 0.0f;
    const typename AC::H h = acc.at(bz, br);
    const float dcr = c1r - c0r, dci = c1i - c0i;
    const double qw = (double)(q * p0.w / g.dt) * 0x1p40;       // charge rate, fixed-point scaled (exact in FP64)
    // J_z flux along z at half nodes bz+ii+1/2 (the last is zero)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        const float B0 = fmaf(0.5f, db[jj], b0[jj]);                // b0 + db/2
        const float B1 = fmaf(1.0f / 3.0f, db[jj], 0.5f * b0[jj]);  // b0/2 + db/3
        const float xr = fmaf(B0, c0r, B1 * dcr), xi = fmaf(B0, c0i, B1 * dci);
        float run0 = 0.0f, runr = 0.0f, runi = 0.0f;
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
            run0 = fmaf(da[ii], B0, run0);
            runr = fmaf(da[ii], xr, runr);
            runi = fmaf(da[ii], xi, runi);
            acc.add(h, 0, ii, jj, fix_mul(-qw, run0));
            acc.add(h, 1, ii, jj, fix_mul(-qw, runr));
            acc.add(h, 2, ii, jj, fix_mul(-qw, runi));
        }
    }
    // J_r flux along r at half nodes br+jj+1/2 (the last is zero)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
        const float A0 = fmaf(0.5f, da[ii], a0[ii]);
        const float A1 = fmaf(1.0f / 3.0f, da[ii], 0.5f * a0[ii]);
        const float xr = fmaf(A0, c0r, A1 * dcr), xi = fmaf(A0, c0i, A1 * dci);
        float run0 = 0.0f, runr = 0.0f, runi = 0.0f;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            run0 = fmaf(db[jj], A0, run0);
            runr = fmaf(db[jj], xr, runr);
            runi = fmaf(db[jj], xi, runi);
            acc.add(h, 3, ii, jj, fix_mul(-qw, run0));
            acc.add(h, 4, ii, jj, fix_mul(-qw, runr));
            acc.add(h, 5, ii, jj, fix_mul(-qw, runi));
        }
    }
    // m 1 azimuthal charge rate W_th (off the axis)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        if (br + jj == 0) continue;
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
            const float wgt = fmaf(da[ii] * db[jj], 1.0f / 3.0f,
                                   fmaf(0.5f * a0[ii], db[jj], fmaf(0.5f * da[ii], b0[jj], a0[ii] * b0[jj])));
            acc.add(h, 7, ii, jj, fix_mul(qw, dcr * wgt));
            acc.add(h, 8, ii, jj, fix_mul(qw, dci * wgt));
        }
    }
    // m 0 azimuthal current at the midpoint: q w v_th with the midpoint shapes
    const float xm = 0.5f * (p0.x + p1.x), ym = 0.5f * (p0.y + p1.y);
    float rm, sm;
    int Km;
    circ_rcell(xm, ym, g.inv_dr, rm, Km, sm);
    if (rm > 0.0f) {
        const float gi = 1.0f / sqrtf(fmaf(p1.u[0], p1.u[0], fmaf(p1.u[1], p1.u[1], fmaf(p1.u[2], p1.u[2], 1.0f))));
        const float vth = (xm * p1.u[1] - ym * p1.u[0]) / rm * gi;
        const float zc = 0.5f * ((p0.oz + (float)carry) + p1.oz);     // midpoint in cells from p0.iz
        const float fz = floorf(zc);
        const int izm = p0.iz + (int)fz;
        const float oz = zc - fz;
        const float fm = circ_fr(Km, sm);
        const float wzz[2] = {1.0f - oz, oz}, wrr[2] = {1.0f - fm, fm};
        const typename AC::H hm = acc.at(izm, Km);
        const double qv = (double)(q * p0.w) * 0x1p40;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) acc.add(hm, 6, a, b, fix_mul(qv, vth * (wzz[a] * wrr[b])));
    }
}

// Removed at the end of its step: a particle that reached the radial wall
// margin (r >= (nr - wall) dr).
__device__ __forceinline__ bool circ_removed(const CircGeom& g, const CircParticle& p) {
    return p.jr >= g.nr - g.wall;
}

// Removed before its step: a particle outside window z cells [kill, nz - 1 - kill]
// (after the window's move at the end of the previous step); it neither moves
// nor deposits, exactly as if removed at the end of that step.
__device__ __forceinline__ bool circ_zkilled(const CircGeom& g, int iz) {
    if (!g.window) return false;
    const int w = circ_zwin(g, iz);
    return w < g.kill || w > g.nz - 1 - g.kill;
}

__device__ __forceinline__ void load_particle(const SpeciesDev& s, int i, int nz, CircParticle& p) {
    const int cl = s.cell[i];
    p.iz = cl % nz;
    p.jr = cl / nz;
    p.oz = s.off[0][i];
    p.x = s.off[1][i];
    p.y = s.off[2][i];
    p.u[0] = s.u[0][i];
    p.u[1] = s.u[1][i];
    p.u[2] = s.u[2][i];
    p.w = s.w[i];
}

// The raw SoA values of particle i (cell, z offset, x, y, u, w).
__device__ __forceinline__ void load_raw(const SpeciesDev& s, int i, int& cell, float o[3], float u[3], float& w) {
    cell = s.cell[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        o[d] = s.off[d][i];
        u[d] = s.u[d][i];
    }
    w = s.w[i];
}

__device__ __forceinline__ void store_particle(const SpeciesDev& s, int i, const CircGeom& g, const CircParticle& p,
                                               bool removed) {
    s.cell[i] = removed ? -1 : p.iz + g.nz * p.jr;
    s.off[0][i] = p.oz;
    s.off[1][i] = p.x;
    s.off[2][i] = p.y;
    s.u[0][i] = p.u[0];
    s.u[1][i] = p.u[1];
    s.u[2][i] = p.u[2];
}

__device__ __forceinline__ void flag(int* err, int e) {
    if (e) atomicOr(err, e);
}

// ------------------------------------------------------------------ split kernels

__global__ void __launch_bounds__(256) k_circ_gather_push(CircGeom g, CircFields F, SpeciesDev s, PrevDev prev,
                                                          const int* __restrict__ d_count, int* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *d_count) return;
    const int cl = s.cell[i];
    if (cl < 0 || circ_zkilled(g, cl % g.nz)) {
        prev.cell[i] = -1;
        if (cl >= 0) s.cell[i] = -1;
        return;
    }
    prev.cell[i] = cl;
    CircParticle p0, p1;
    load_particle(s, i, g.nz, p0);
    prev.off[0][i] = p0.oz;
    prev.off[1][i] = p0.x;
    prev.off[2][i] = p0.y;
    const GField fa{&g, &F};
    const int e = circ_push(g, fa, s.qmh, p0, p1);
    flag(err, e);
    store_particle(s, i, g, p1, circ_removed(g, p1));
    if (circ_removed(g, p1)) s.cell[i] = -2 - (p1.iz + g.nz * (p1.jr < g.nr ? p1.jr : g.nr - 1));
}

// Deposit of x^n (prev) -> x^{n+1} (s); particles marked -2 - cell moved out
// this step and still deposit.
__global__ void __launch_bounds__(256) k_circ_deposit(CircGeom g, SpeciesDev s, PrevDev prev,
                                                      const int* __restrict__ d_count, float q,
                                                      unsigned long long* acc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *d_count) return;
    const int c0 = prev.cell[i];
    if (c0 < 0) return;
    CircParticle p0, p1;
    p0.iz = c0 % g.nz;
    p0.jr = c0 / g.nz;
    p0.oz = prev.off[0][i];
    p0.x = prev.off[1][i];
    p0.y = prev.off[2][i];
    p0.w = s.w[i];
    int c1 = s.cell[i];
    if (c1 < 0) c1 = -2 - c1;
    p1.iz = c1 % g.nz;
    p1.jr = c1 / g.nz;
    p1.oz = s.off[0][i];
    p1.x = s.off[1][i];
    p1.y = s.off[2][i];
    p1.u[0] = s.u[0][i];
    p1.u[1] = s.u[1][i];
    p1.u[2] = s.u[2][i];
    p1.w = p0.w;
    const GAcc ac{acc, g.nz, g.ncell};
    circ_deposit(g, ac, q, p0, p1);
}

// After a split deposit: particles marked -2 - cell become removed (-1).
__global__ void k_circ_finalize_removed(int* cell, const int* __restrict__ d_count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *d_count) return;
    if (cell[i] <= -2) cell[i] = -1;
}

// ------------------------------------------------------------------ fused tiled kernel

// Tile of workgroup b: chunks of `chunk` consecutive tiles go round-robin
// to the 8 XCDs (consecutive workgroup indices run on consecutive XCDs);
// -1 past the last tile.  The launch has circ_xcd_blocks(ntiles, chunk)
// workgroups.
__device__ __forceinline__ int circ_xcd_tile(int b, int ntiles, int chunk) {
    const int k = b % 8, j = b / 8;
    const long long tile = (long long)(k + 8 * (j / chunk)) * chunk + j % chunk;
    return tile < ntiles ? (int)tile : -1;
}

inline int circ_xcd_blocks(int ntiles, int chunk) {
    const int nchunks = (ntiles + chunk - 1) / chunk;
    return 8 * ((nchunks + 7) / 8) * chunk;
}

template <int TZ, int TR, int G>
struct CircTile {
    static constexpr int SZ = TZ + 2 * G + 2, SR = TR + 2 * G + 2;       // staged field nodes
    static constexpr int AZ = TZ + 2 * G + 3, AR = TR + 2 * G + 3;       // current nodes
    static constexpr size_t kFieldFloats = 18 * (size_t)SZ * SR;
    static constexpr size_t kAccWords = (size_t)kCircChannels * AZ * AR;
    static constexpr size_t kLds = kFieldFloats * 4 + kAccWords * 8;
};

// One workgroup per tile of TZ x TR cells.  toff: tile ranges of the last
// sort (tiles z-fastest: tile = tz + ntz * tr).  Particles outside the tile's
// guard are appended to the rest list.
template <int TZ, int TR, int G, int NT>
__global__ void __launch_bounds__(NT) k_circ_tile(CircGeom g, CircFields F, SpeciesDev s,
                                                   const int* __restrict__ toff, int ntz, int ntiles,
                                                   unsigned long long* gacc, int* err, int* rest_n, int* rest_idx) {
    using T = CircTile<TZ, TR, G>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float* fl = reinterpret_cast<float*>(lds_raw);
    unsigned long long* al = reinterpret_cast<unsigned long long*>(lds_raw + T::kFieldFloats * 4);
    // rows of tiles along z dealt round-robin to the 8 XCDs (neighbours in a
    // row share their halos in one L2)
    const int tile = circ_xcd_tile(blockIdx.x, ntiles, ntz);
    if (tile < 0) return;
    const int tz = tile % ntz, tr = tile / ntz;
    const int z0 = tz * TZ, r0 = tr * TR;
    const int p_begin = toff[tile], p_end = toff[tile + 1];
    if (p_begin == p_end) return;
    // stage fields: z [z0 - G - 1, z0 + TZ + G], r [r0 - G - 1, r0 + TR + G]
    const int fz0 = z0 - G - 1, fr0 = r0 - G - 1;
    for (int k = threadIdx.x; k < 18 * T::SZ * T::SR; k += blockDim.x) {
        const int plane = k / (T::SZ * T::SR);
        const int rem = k - plane * (T::SZ * T::SR);
        const int jr = fr0 + rem / T::SZ;
        int iz = fz0 + rem % T::SZ;
        iz = iz < 0 ? iz + g.nz : (iz >= g.nz ? iz - g.nz : iz);
        const int f = plane / 9, c = (plane / 3) % 3, ch = plane % 3;
        float v = 0.0f;
        if (jr >= 0 && jr < g.nr) {
            v = F.F[f][c][ch][iz + g.nz * jr];
        }
        fl[k] = v;
    }
    for (int k = threadIdx.x; k < (int)T::kAccWords; k += blockDim.x) al[k] = 0ull;
    __syncthreads();
    const LField lf{fl, (fz0 % g.nz + g.nz) % g.nz, fr0, g.nz, T::SZ, T::SR};
    const LAcc la{al, ((z0 - G - 1) % g.nz + g.nz) % g.nz, r0 - G - 1, g.nz, T::AZ, T::AR};
    const float q = -s.mq;
    int e = 0;
    // software pipeline: the next particle's SoA loads are issued before the
    // current particle is processed
    int i = p_begin + (int)threadIdx.x;
    int cn = -1;
    float on[3] = {0.f, 0.f, 0.f}, un[3] = {0.f, 0.f, 0.f}, wn = 0.f;
    if (i < p_end) load_raw(s, i, cn, on, un, wn);
    for (; i < p_end; i += NT) {
        const int cl = cn;
        CircParticle p0, p1;
        p0.iz = cl % g.nz;
        p0.jr = cl / g.nz;
        p0.oz = on[0];
        p0.x = on[1];
        p0.y = on[2];
        p0.u[0] = un[0];
        p0.u[1] = un[1];
        p0.u[2] = un[2];
        p0.w = wn;
        if (i + NT < p_end) load_raw(s, i + NT, cn, on, un, wn);
        if (cl < 0) continue;
        if (circ_zkilled(g, p0.iz)) {
            s.cell[i] = -1;
            continue;
        }
        int dz = p0.iz - z0;
        if (dz < -G) dz += g.nz;
        else if (dz >= g.nz - G) dz -= g.nz;
        // the radial cell the stencils use is recomputed from (x, y): test that one
        float rr, ss;
        int K;
        circ_rcell(p0.x, p0.y, g.inv_dr, rr, K, ss);
        const int dr = K - r0;
        if (dz < -G || dz >= TZ + G || dr < -G || dr >= TR + G) {
            rest_idx[atomicAdd(rest_n, 1)] = i;
            continue;
        }
        const int ef = circ_push(g, lf, s.qmh, p0, p1);
        e |= ef;
        circ_deposit(g, la, q, p0, p1);
        store_particle(s, i, g, p1, circ_removed(g, p1));
    }
    flag(err, e);
    __syncthreads();
    // flush: the tile's current into the global accumulator
    for (int k = threadIdx.x; k < (int)T::kAccWords; k += blockDim.x) {
        const unsigned long long v = al[k];
        if (!v) continue;
        const int ch = k / (T::AZ * T::AR);
        const int rem = k - ch * (T::AZ * T::AR);
        const int jr = r0 - G - 1 + rem / T::AZ;
        int iz = z0 - G - 1 + rem % T::AZ;
        iz = iz < 0 ? iz + g.nz : (iz >= g.nz ? iz - g.nz : iz);
        if (jr < 0 || jr >= g.nr) continue;
        atomicAdd(gacc + (size_t)ch * g.ncell + iz + g.nz * jr, v);
    }
}

// Rest pass: the rest list of the last tile launch and the particles appended
// after the last sort, through global memory.
__global__ void __launch_bounds__(256) k_circ_rest(CircGeom g, CircFields F, SpeciesDev s,
                                                   const int* __restrict__ d_sorted, const int* __restrict__ d_count,
                                                   const int* __restrict__ rest_n, const int* __restrict__ rest_idx,
                                                   unsigned long long* gacc, int* err) {
    const int nrest = *rest_n;
    const int sorted = *d_sorted, count = *d_count;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    int i;
    if (k < nrest) i = rest_idx[k];
    else if (k - nrest < count - sorted) i = sorted + (k - nrest);
    else return;
    const int cl = s.cell[i];
    if (cl < 0) return;
    if (circ_zkilled(g, cl % g.nz)) {
        s.cell[i] = -1;
        return;
    }
    CircParticle p0, p1;
    load_particle(s, i, g.nz, p0);
    const GField fa{&g, &F};
    const int ef = circ_push(g, fa, s.qmh, p0, p1);
    flag(err, ef);
    const GAcc ac{gacc, g.nz, g.ncell};
    circ_deposit(g, ac, -s.mq, p0, p1);
    store_particle(s, i, g, p1, circ_removed(g, p1));
}

__global__ void k_circ_zero_rest(int* rest_n) { *rest_n = 0; }

// ------------------------------------------------------------------ current read-out

// acc (2^-40 units) -> J planes [3 comps][3 channels], with the node geometry:
// J_z = flux dz / V_j, J_r = flux / (2 pi r_{j+1/2} dz), J_th m1 = -i r_j rate / V_j,
// J_th m0 = acc / V_j; on the axis J_th m1 = -i J_r m1 (dr/2).  Zeroes acc if asked.
__global__ void __launch_bounds__(256) k_circ_jfinal(CircGeom g, unsigned long long* acc, float* Jz0, float* Jz1,
                                                     float* Jz2, float* Jr0, float* Jr1, float* Jr2, float* Jt0,
                                                     float* Jt1, float* Jt2, int zero) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ncell) return;
    const int j = idx / g.nz;
    const double pi = 3.14159265358979323846;
    const double dr = g.dr, dz = g.dz;
    const double V = j == 0 ? pi * 0.25 * dr * dr * dz : 2.0 * pi * (double)j * dr * dr * dz;
    const double Ah = 2.0 * pi * ((double)j + 0.5) * dr * dz;
    double a[kCircChannels];
#pragma unroll
    for (int c = 0; c < kCircChannels; ++c) a[c] = (double)(long long)acc[(size_t)c * g.ncell + idx] * PIC_FIX_INV;
    Jz0[idx] = (float)(a[0] * dz / V);
    Jz1[idx] = (float)(a[1] * dz / V);
    Jz2[idx] = (float)(a[2] * dz / V);
    Jr0[idx] = (float)(a[3] / Ah);
    Jr1[idx] = (float)(a[4] / Ah);
    Jr2[idx] = (float)(a[5] / Ah);
    Jt0[idx] = (float)(a[6] / V);
    if (j == 0) {
        // -i J_r(dr/2) of m 1, J_r at this node's half node (j + 1/2 = 1/2)
        Jt1[idx] = (float)(a[5] / Ah);
        Jt2[idx] = (float)(-a[4] / Ah);
    } else {
        const double rj = (double)j * dr;
        Jt1[idx] = (float)(rj * a[8] / V);    // -i (a + i b) = b - i a
        Jt2[idx] = (float)(-rj * a[7] / V);
    }
    if (zero) {
#pragma unroll
        for (int c = 0; c < kCircChannels; ++c) acc[(size_t)c * g.ncell + idx] = 0ull;
    }
}

// ------------------------------------------------------------------ field update

// Storage z neighbours across the window: valid unless beyond the window's ends.
struct ZNb {
    int im, ip;
    bool okm, okp;
};

__device__ __forceinline__ ZNb znb(const CircGeom& g, int i) {
    ZNb n;
    n.im = i == 0 ? g.nz - 1 : i - 1;
    n.ip = i == g.nz - 1 ? 0 : i + 1;
    const int w = circ_zwin(g, i);
    n.okm = g.window ? w > 0 : i > 0;
    n.okp = g.window ? w < g.nz - 1 : i < g.nz - 1;
    return n;
}

struct CircFieldsRW {
    float* F[2][3][3];   // E, B: [comp z, r, th][channel m0, Re m1, Im m1]
};

struct CircJ {
    const float* J[9];   // [comp z, r, th][channel]
};

// B -= h curl E for both modes at node (i, j) (storage z).
__global__ void __launch_bounds__(256) k_circ_bhalf(CircGeom g, CircFieldsRW F, float h) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ncell) return;
    const int j = idx / g.nz, i = idx - j * g.nz;
    const ZNb n = znb(g, i);
    const float dr = g.dr;
    const float rh = ((float)j + 0.5f) * dr;
    const bool top = j + 1 >= g.nr;
    for (int ch = 0; ch < 3; ++ch) {
        const float m = ch == 0 ? 0.0f : 1.0f;
        const float* Ez = F.F[0][0][ch];
        const float* Er = F.F[0][1][ch];
        const float* Et = F.F[0][2][ch];
        // the partner channel for the i m / r terms: i (a + i b) = -b + i a
        const int pc = ch == 1 ? 2 : 1;
        const float ps = ch == 1 ? -1.0f : 1.0f;
        const float* Ezp = F.F[0][0][pc];
        const float* Erp = F.F[0][1][pc];
        // (curl E)_z at (i, j+1/2) = (1/r) d_r (r E_th) + (i m / r) E_r
        const float etu = top ? 0.0f : Et[idx + g.nz];
        float cz = ((float)(j + 1) * dr * etu - (float)j * dr * Et[idx]) / (rh * dr);
        if (ch) cz += ps * Erp[idx] / rh;
        // (curl E)_r at (i+1/2, j) = -(i m / r) E_z - d_z E_th
        const float etp = n.okp ? Et[j * g.nz + n.ip] : 0.0f;
        float cr;
        if (j == 0) {
            if (ch == 0) {
                cr = 0.0f;
            } else {
                const float ezu = g.nr > 1 ? Ezp[idx + g.nz] : 0.0f;
                cr = -(ps * ezu) / dr - (etp - Et[idx]) / g.dz;
            }
        } else {
            cr = (ch ? -(ps * Ezp[idx]) / ((float)j * dr) : 0.0f) - (etp - Et[idx]) / g.dz;
        }
        // (curl E)_th at (i+1/2, j+1/2) = d_z E_r - d_r E_z
        const float erp = n.okp ? Er[j * g.nz + n.ip] : 0.0f;
        const float ezu = top ? 0.0f : Ez[idx + g.nz];
        const float ct = (erp - Er[idx]) / g.dz - (ezu - Ez[idx]) / dr;
        (void)m;
        // defer the writes until every channel's E has been read: E is not written here
        F.F[1][0][ch][idx] -= h * cz;
        F.F[1][1][ch][idx] = (j == 0 && ch == 0) ? 0.0f : F.F[1][1][ch][idx] - h * cr;
        F.F[1][2][ch][idx] -= h * ct;
    }
}

// E += dt (curl B - J) for both modes at node (i, j).
__global__ void __launch_bounds__(256) k_circ_efull(CircGeom g, CircFieldsRW F, CircJ Jp) {
    const float* const* J = Jp.J;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ncell) return;
    const int j = idx / g.nz, i = idx - j * g.nz;
    const ZNb n = znb(g, i);
    const float dr = g.dr;
    const float rh = ((float)j + 0.5f) * dr;
    for (int ch = 0; ch < 3; ++ch) {
        const float* Bz = F.F[1][0][ch];
        const float* Br = F.F[1][1][ch];
        const float* Bt = F.F[1][2][ch];
        const int pc = ch == 1 ? 2 : 1;
        const float ps = ch == 1 ? -1.0f : 1.0f;
        const float* Bzp = F.F[1][0][pc];
        const float* Brp = F.F[1][1][pc];
        // (curl B)_z at (i+1/2, j) = (1/r) d_r (r B_th) + (i m / r) B_r
        float cz;
        if (j == 0) {
            cz = ch == 0 ? 4.0f * Bt[idx] / dr : 0.0f;
        } else {
            const float rj = (float)j * dr;
            cz = (rh * Bt[idx] - (rh - dr) * Bt[idx - g.nz]) / (rj * dr);
            if (ch) cz += ps * Brp[idx] / rj;
        }
        // (curl B)_r at (i, j+1/2) = -(i m / r) B_z - d_z B_th
        const float btm = n.okm ? Bt[j * g.nz + n.im] : 0.0f;
        float cr = -(Bt[idx] - btm) / g.dz;
        if (ch) cr -= ps * Bzp[idx] / rh;
        // (curl B)_th at (i, j) = d_z B_r - d_r B_z
        const float brm = n.okm ? Br[j * g.nz + n.im] : 0.0f;
        float ct;
        if (j == 0) {
            ct = ch == 0 ? 0.0f : (Br[idx] - brm) / g.dz - 2.0f * Bz[idx] / dr;
        } else {
            ct = (Br[idx] - brm) / g.dz - (Bz[idx] - Bz[idx - g.nz]) / dr;
        }
        float* Ez = F.F[0][0][ch];
        float* Er = F.F[0][1][ch];
        float* Et = F.F[0][2][ch];
        const float jz = J[0 * 3 + ch][idx], jr = J[1 * 3 + ch][idx], jt = J[2 * 3 + ch][idx];
        Ez[idx] = (j == 0 && ch != 0) ? 0.0f : Ez[idx] + g.dt * (cz - jz);
        Er[idx] = Er[idx] + g.dt * (cr - jr);
        Et[idx] = (j == 0 && ch == 0) ? 0.0f : Et[idx] + g.dt * (ct - jt);
    }
}

// Total-field / scattered-field corrections of the mode-1 laser (E_x = B_y):
// plane iz of the B planes (which 0) or the E planes (which 1).
__global__ void k_circ_laser(CircGeom g, CircFieldsRW F, int iz, int which, double coef, double inv_w2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.nr) return;
    const double rj = (double)j * g.dr, rh = ((double)j + 0.5) * g.dr;
    const float fj = (float)(coef * exp(-rj * rj * inv_w2));
    const float fh = (float)(coef * exp(-rh * rh * inv_w2));
    const int idx = iz + g.nz * j;
    if (which == 0) {
        F.F[1][2][1][idx] += fh;      // B_th += h e f / dz
        F.F[1][1][2][idx] += fj;      // B_r  += i h e f / dz
    } else {
        F.F[0][1][1][idx] += fh;      // E_r  += dt e f / dz
        F.F[0][2][2][idx] -= fj;      // E_th += -i dt e f / dz
    }
}

// Window motion: zero the plane at storage z `iz` of all 18 field planes.
__global__ void k_circ_clear_plane(CircGeom g, CircFieldsRW F, int iz) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 18 * g.nr) return;
    const int plane = k / g.nr, j = k - plane * g.nr;
    const int f = plane / 9, c = (plane / 3) % 3, ch = plane % 3;
    F.F[f][c][ch][iz + g.nz * j] = 0.0f;
}

// ------------------------------------------------------------------ plasma loading

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed, unsigned long long k) {
    unsigned long long z = seed * 0x9E3779B97F4A7C15ull + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform53(unsigned long long seed, unsigned long long k) {
    return (double)(splitmix64(seed, k) >> 11) * 0x1p-53;
}

// Particle (window z cell zb + a, radial cell j, slot s): counter
// c = ((Z nr + j) ppc + s), Z = lab cell; draws 3c, 3c+1, 3c+2 of the stream.
__global__ void __launch_bounds__(256) k_circ_inject(CircGeom g, SpeciesDev s, long long shift, int zb, int nzs,
                                                     int r_cells, int ppc, unsigned long long seed, double z_start,
                                                     double ramp, double n_plateau, double dz, double dr,
                                                     int* d_count, int capacity, int* err) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)nzs * r_cells * ppc;
    if (k >= total) return;
    const int sl = (int)(k % ppc);
    const int j = (int)((k / ppc) % r_cells);
    const int a = (int)(k / ((long long)ppc * r_cells));
    const long long Z = (long long)(zb + a) + shift;
    const unsigned long long c = (unsigned long long)((Z * g.nr + j) * ppc + sl);
    const double uz = uniform53(seed, 3ull * c);
    const double ur = uniform53(seed, 3ull * c + 1ull);
    const double ut = uniform53(seed, 3ull * c + 2ull);
    const float oz = (float)(floor(uz * 0x1p24) * 0x1p-24);
    const double r = ((double)j + ur) * dr;
    const double th = 6.283185307179586 * ut;
    const double zl = ((double)Z + (double)oz) * dz;
    double n = 0.0;
    if (zl >= z_start) n = zl < z_start + ramp ? n_plateau * (zl - z_start) / (ramp > 0.0 ? ramp : 1e-300) : n_plateau;
    if (!(n > 0.0)) return;
    const int at = atomicAdd(d_count, 1);
    if (at >= capacity) {
        atomicOr(err, ERR_OVERFLOW);
        return;
    }
    const float x = (float)(r * cos(th)), y = (float)(r * sin(th));
    int iz = zb + a + (g.window ? g.origin : 0);
    if (iz >= g.nz) iz -= g.nz;
    float rr, ss;
    int K;
    circ_rcell(x, y, g.inv_dr, rr, K, ss);
    s.cell[at] = iz + g.nz * K;
    s.off[0][at] = oz;
    s.off[1][at] = x;
    s.off[2][at] = y;
    s.u[0][at] = 0.0f;
    s.u[1][at] = 0.0f;
    s.u[2][at] = 0.0f;
    s.w[at] = (float)(n * 2.0 * 3.14159265358979323846 * r * dr * dz / ppc);
    s.id[at] = (int)(c & 0x7FFFFFFFull);
}

// ------------------------------------------------------------------ diagnostics

// out[0] += sum q w, out[1] += sum m w (gamma - 1), cnt += live
__global__ void __launch_bounds__(256) k_circ_diag_particles(CircGeom g, SpeciesDev s, const int* d_count, double q,
                                                             double m, double* out, unsigned long long* cnt) {
    double a = 0.0, b = 0.0;
    unsigned long long live = 0;
    const int n = *d_count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int cl = s.cell[i];
        if (cl < 0 || circ_zkilled(g, cl % g.nz)) continue;
        const double ux = s.u[0][i], uy = s.u[1][i], uz = s.u[2][i];
        const double u2 = ux * ux + uy * uy + uz * uz;
        a += q * (double)s.w[i];
        b += m * (double)s.w[i] * (u2 / (sqrt(1.0 + u2) + 1.0));
        ++live;
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        live += __shfl_xor(live, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out + 0, a);
        atomicAdd(out + 1, b);
        atomicAdd(cnt, live);
    }
}

// out[2] += field energy: sum V (|F_0|^2 + |F_1|^2 / 2) / 2, half-r components with 2 pi r_{j+1/2} dr dz
__global__ void __launch_bounds__(256) k_circ_diag_fields(CircGeom g, CircFields F, CircJ J, double* out,
                                                          unsigned int* jmax) {
    double e = 0.0;
    float mj = 0.0f;
    const double pi = 3.14159265358979323846;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.ncell; idx += gridDim.x * blockDim.x) {
        const int j = idx / g.nz;
        const double Vi = j == 0 ? pi * 0.25 * g.dr * g.dr * g.dz : 2.0 * pi * (double)j * g.dr * g.dr * g.dz;
        const double Vh = 2.0 * pi * ((double)j + 0.5) * g.dr * g.dr * g.dz;
        for (int f = 0; f < 2; ++f)
            for (int c = 0; c < 3; ++c) {
                const bool half = f == 0 ? c == 1 : c != 1;
                const double V = half ? Vh : Vi;
                const double a = F.F[f][c][0][idx], b = F.F[f][c][1][idx], d = F.F[f][c][2][idx];
                e += 0.5 * V * (a * a + 0.5 * (b * b + d * d));
            }
        for (int k = 0; k < 9; ++k) mj = fmaxf(mj, fabsf(J.J[k][idx]));
    }
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o, 64);
        mj = fmaxf(mj, __shfl_xor(mj, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out + 2, e);
        atomicMax(jmax, __float_as_uint(mj));
    }
}

int grid1(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

// ------------------------------------------------------------------ launchers

constexpr int kCircTZ = 32, kCircTR = 8, kCircG = 1;

size_t circ_tile_lds() { return CircTile<kCircTZ, kCircTR, kCircG>::kLds; }
int circ_tile_z() { return kCircTZ; }
int circ_tile_r() { return kCircTR; }

hipError_t launch_circ_gather_push(const CircGeom& g, const CircFields& F, const SpeciesDev& s, const PrevDev& prev,
                                   const int* d_count, int max_count, int* err, hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_circ_gather_push, dim3(grid1(max_count)), dim3(256), 0, st, g, F, s, prev, d_count, err);
    return hipGetLastError();
}

hipError_t launch_circ_deposit(const CircGeom& g, const SpeciesDev& s, const PrevDev& prev, const int* d_count,
                               int max_count, float q, unsigned long long* acc, hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_circ_deposit, dim3(grid1(max_count)), dim3(256), 0, st, g, s, prev, d_count, q, acc);
    hipLaunchKernelGGL(k_circ_finalize_removed, dim3(grid1(max_count)), dim3(256), 0, st, s.cell, d_count);
    return hipGetLastError();
}

template <int NT>
hipError_t launch_circ_tile_nt(const CircGeom& g, const CircFields& F, const SpeciesDev& s, const int* toff, int ntz,
                               int ntiles, unsigned long long* acc, int* err, int* rest_n, int* rest_idx,
                               hipStream_t st) {
    using T = CircTile<kCircTZ, kCircTR, kCircG>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_circ_tile<kCircTZ, kCircTR, kCircG, NT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)T::kLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_circ_tile<kCircTZ, kCircTR, kCircG, NT>), dim3(circ_xcd_blocks(ntiles, ntz)), dim3(NT),
                       T::kLds, st, g, F, s, toff, ntz, ntiles, acc, err, rest_n, rest_idx);
    return hipGetLastError();
}

hipError_t launch_circ_tile(const CircGeom& g, const CircFields& F, const SpeciesDev& s, const int* toff, int ntz,
                            int ntiles, unsigned long long* acc, int* err, int* rest_n, int* rest_idx, int threads,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_circ_zero_rest, dim3(1), dim3(1), 0, st, rest_n);
    switch (threads) {
        case 256: return launch_circ_tile_nt<256>(g, F, s, toff, ntz, ntiles, acc, err, rest_n, rest_idx, st);
        case 1024: return launch_circ_tile_nt<1024>(g, F, s, toff, ntz, ntiles, acc, err, rest_n, rest_idx, st);
        default: return launch_circ_tile_nt<512>(g, F, s, toff, ntz, ntiles, acc, err, rest_n, rest_idx, st);
    }
}

hipError_t launch_circ_rest(const CircGeom& g, const CircFields& F, const SpeciesDev& s, const int* d_sorted,
                            const int* d_count, const int* rest_n, const int* rest_idx, int max_items,
                            unsigned long long* acc, int* err, hipStream_t st) {
    if (max_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_circ_rest, dim3(grid1(max_items)), dim3(256), 0, st, g, F, s, d_sorted, d_count, rest_n,
                       rest_idx, acc, err);
    return hipGetLastError();
}

hipError_t launch_circ_jfinal(const CircGeom& g, unsigned long long* acc, float* const J[9], int zero,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_circ_jfinal, dim3(grid1(g.ncell)), dim3(256), 0, st, g, acc, J[0], J[1], J[2], J[3], J[4],
                       J[5], J[6], J[7], J[8], zero);
    return hipGetLastError();
}

hipError_t launch_circ_bhalf(const CircGeom& g, float* const F[2][3][3], float h, hipStream_t st) {
    CircFieldsRW f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) f.F[a][b][c] = F[a][b][c];
    hipLaunchKernelGGL(k_circ_bhalf, dim3(grid1(g.ncell)), dim3(256), 0, st, g, f, h);
    return hipGetLastError();
}

hipError_t launch_circ_efull(const CircGeom& g, float* const F[2][3][3], float* const J[9], hipStream_t st) {
    CircFieldsRW f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) f.F[a][b][c] = F[a][b][c];
    CircJ jj;
    for (int k = 0; k < 9; ++k) jj.J[k] = J[k];
    hipLaunchKernelGGL(k_circ_efull, dim3(grid1(g.ncell)), dim3(256), 0, st, g, f, jj);
    return hipGetLastError();
}

hipError_t launch_circ_laser(const CircGeom& g, float* const F[2][3][3], int iz, int which, double coef,
                             double inv_w2, hipStream_t st) {
    CircFieldsRW f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) f.F[a][b][c] = F[a][b][c];
    hipLaunchKernelGGL(k_circ_laser, dim3(grid1(g.nr)), dim3(256), 0, st, g, f, iz, which, coef, inv_w2);
    return hipGetLastError();
}

hipError_t launch_circ_clear_plane(const CircGeom& g, float* const F[2][3][3], int iz, hipStream_t st) {
    CircFieldsRW f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) f.F[a][b][c] = F[a][b][c];
    hipLaunchKernelGGL(k_circ_clear_plane, dim3(grid1(18 * g.nr)), dim3(256), 0, st, g, f, iz);
    return hipGetLastError();
}

hipError_t launch_circ_inject(const CircGeom& g, const SpeciesDev& s, long long shift, int zb, int ze, int r_cells,
                              int ppc, unsigned long long seed, double z_start, double ramp, double n_plateau,
                              double dz, double dr, int* d_count, int capacity, int* err, hipStream_t st) {
    const long long total = (long long)(ze - zb) * r_cells * ppc;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_circ_inject, dim3(grid1(total)), dim3(256), 0, st, g, s, shift, zb, ze - zb, r_cells, ppc,
                       seed, z_start, ramp, n_plateau, dz, dr, d_count, capacity, err);
    return hipGetLastError();
}

hipError_t launch_circ_diag(const CircGeom& g, const CircFields& F, float* const Jp[9], const SpeciesDev* s,
                            const int* const* d_count, const double* q, const double* m, const int* max_count,
                            int nspecies, double* out, unsigned long long* cnt, unsigned int* jmax, hipStream_t st) {
    for (int k = 0; k < nspecies; ++k) {
        if (max_count[k] <= 0) continue;
        int b = grid1(max_count[k]);
        if (b > 4096) b = 4096;
        hipLaunchKernelGGL(k_circ_diag_particles, dim3(b), dim3(256), 0, st, g, s[k], d_count[k], q[k], m[k], out,
                           cnt);
    }
    int b = grid1(g.ncell);
    if (b > 4096) b = 4096;
    CircJ jj;
    for (int k = 0; k < 9; ++k) jj.J[k] = Jp[k];
    hipLaunchKernelGGL(k_circ_diag_fields, dim3(b), dim3(256), 0, st, g, F, jj, out, jmax);
    return hipGetLastError();
}

}  // namespace pic
