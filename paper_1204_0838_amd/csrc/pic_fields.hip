// FDTD field kernels: the B half step with the (optionally smoothed) curl of E,
// the E step with the standard curl of B and the current, the binomial current
// filter, and small utility kernels.
//
// Boundaries: y and z periodic, or (transverse absorbing layer) zero-valued
// beyond the y and z edges with the layer's stretched derivatives in its
// cells.  x periodic, or (moving window) a circular buffer in which the two
// planes where the window ends meet see zero-valued ghost fields across that
// seam.
//
// The layer (Section 3.1 surrounds the box transversely with a 16-layer
// PML) is the convolutional form: each transverse derivative D of a curl
// inside it is replaced by D + psi with psi <- b psi + (b - 1) D,
// b = exp(-sigma dt), sigma graded over the layer.  The two B half steps of
// a field step together are the leapfrog step of B between half-integer
// times, so the B arrays follow that recursion: the first half step of a
// step advances them with E^n, the second reads the value the next step's
// first half step will store (it sees the same E^{n+1}).
#include <algorithm>

#include "pic_internal.h"

namespace pic {

// Neighbour indices of one cell along each axis with the boundary rule.
struct Nbr {
    int i, j, k;              // cell
    int ip, im, jp, jm, kp, km;  // neighbour coordinates (wrapped)
    bool xp_ok, xm_ok;        // false when the x neighbour lies across the window seam
};

__device__ __forceinline__ Nbr neighbours(const Geom& g, int idx) {
    Nbr n;
    n.k = idx / g.nxy;
    const int r = idx - n.k * g.nxy;
    n.j = r / g.n[0];
    n.i = r - n.j * g.n[0];
    n.ip = n.i + 1 == g.n[0] ? 0 : n.i + 1;
    n.im = n.i == 0 ? g.n[0] - 1 : n.i - 1;
    n.jp = n.j + 1 == g.n[1] ? 0 : n.j + 1;
    n.jm = n.j == 0 ? g.n[1] - 1 : n.j - 1;
    n.kp = n.k + 1 == g.n[2] ? 0 : n.k + 1;
    n.km = n.k == 0 ? g.n[2] - 1 : n.k - 1;
    n.xp_ok = true;
    n.xm_ok = true;
    if (g.window) {
        int xw = n.i - g.origin;
        if (xw < 0) xw += g.n[0];
        n.xp_ok = xw != g.n[0] - 1;
        n.xm_ok = xw != 0;
    }
    return n;
}

__device__ __forceinline__ int at(const Geom& g, int i, int j, int k) { return i + g.n[0] * (j + g.n[1] * k); }

// B -= h curl' E with forward differences, curl'_x = D_y S_y E_z - D_z S_z E_y
// (cyclic), where S_axis is the transverse smoothing of the Section 2 stencil
// (identity for the Yee scheme): centre alpha_axis, +-t1 neighbours beta_t1,
// +-t2 neighbours beta_t2, the four corners gamma_{t1 t2}, t1 = axis + 1 and
// t2 = axis + 2 cyclically.  y and z are periodic; with the moving window,
// x neighbours across the window seam read as zero.
//
// LDS-tiled: E is staged on a tile of BT_X x BT_Y x BT_Z cells plus a
// one-cell halo, in window coordinates, with zeros beyond the window's two
// ends (or periodic images without a window), so a neighbour across the seam
// is exactly a zero-filled halo cell.
constexpr int BT_X = 32, BT_Y = 8, BT_Z = 4, BT_THREADS = 256;
constexpr int BS_X = BT_X + 2, BS_Y = BT_Y + 2, BS_Z = BT_Z + 2, BS_N = BS_X * BS_Y * BS_Z;

template <int AXIS>
__device__ __forceinline__ float smooth_l(const PDCoef& c, const float* F, int o) {
    constexpr int X = 1, Y = BS_X, Z = BS_X * BS_Y;
    const float ctr = F[o];
    if (AXIS == 0) {
        const float ny = F[o + Y] + F[o - Y];
        const float nz = F[o + Z] + F[o - Z];
        const float cr = (F[o + Y + Z] + F[o - Y + Z]) + (F[o + Y - Z] + F[o - Y - Z]);
        return fmaf(c.gam[0], cr, fmaf(c.beta[2], nz, fmaf(c.beta[1], ny, c.alpha[0] * ctr)));
    } else if (AXIS == 1) {
        const float nz = F[o + Z] + F[o - Z];
        const float nx = F[o + X] + F[o - X];
        const float cr = (F[o + X + Z] + F[o - X + Z]) + (F[o + X - Z] + F[o - X - Z]);
        return fmaf(c.gam[1], cr, fmaf(c.beta[0], nx, fmaf(c.beta[2], nz, c.alpha[1] * ctr)));
    } else {
        const float nx = F[o + X] + F[o - X];
        const float ny = F[o + Y] + F[o - Y];
        const float cr = (F[o + X + Y] + F[o - X + Y]) + (F[o + X - Y] + F[o - X - Y]);
        return fmaf(c.gam[2], cr, fmaf(c.beta[1], ny, fmaf(c.beta[0], nx, c.alpha[2] * ctr)));
    }
}

template <bool PD, int AXIS>
__device__ __forceinline__ float sval_l(const PDCoef& c, const float* F, int o) {
    if (PD) return smooth_l<AXIS>(c, F, o);
    return F[o];
}

// psi' = b psi + (b - 1) D (stored when `store`), returns D + psi'.
__device__ __forceinline__ float pml_stretch(float* __restrict__ psi, size_t q, float b, float bm1, float D,
                                             bool store) {
    const float p = fmaf(b, psi[q], bm1 * D);
    if (store) psi[q] = p;
    return D + p;
}

// One tile (tile coordinates bx, by, bz) of the LDS-tiled B half step.
template <bool PD, bool PML>
__device__ __forceinline__ void bhalf_tile(const Geom& g, const PDCoef& c, const float* __restrict__ Ex,
                                           const float* __restrict__ Ey, const float* __restrict__ Ez,
                                           float* __restrict__ Bx, float* __restrict__ By, float* __restrict__ Bz,
                                           float h, int bx, int by, int bz, float (*El)[BS_N], const PmlDev& P,
                                           bool store) {
    const int t0[3] = {bx * BT_X, by * BT_Y, bz * BT_Z};
    const int origin = g.window ? g.origin : 0;
    constexpr int PER = (BS_N + BT_THREADS - 1) / BT_THREADS;
    float v[PER][3];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * BT_THREADS;
        const int hx = i % BS_X, r = i / BS_X, hy = r % BS_Y, hz = r / BS_Y;
        int xw = t0[0] - 1 + hx, y = t0[1] - 1 + hy, z = t0[2] - 1 + hz;
        bool ok = i < BS_N;
        if (PML) ok = ok && y >= 0 && y < g.n[1] && z >= 0 && z < g.n[2];   // zero beyond the edges
        y = ((y % g.n[1]) + g.n[1]) % g.n[1];
        z = ((z % g.n[2]) + g.n[2]) % g.n[2];
        if (g.window) {
            ok = ok && xw >= 0 && xw < g.n[0];
        } else {
            xw = ((xw % g.n[0]) + g.n[0]) % g.n[0];
        }
        int xs = xw + origin;
        xs = xs >= g.n[0] ? xs - g.n[0] : xs;
        const int s = xs + g.n[0] * (y + g.n[1] * z);
        v[q][0] = ok ? Ex[s] : 0.0f;
        v[q][1] = ok ? Ey[s] : 0.0f;
        v[q][2] = ok ? Ez[s] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * BT_THREADS;
        if (i < BS_N) {
            El[0][i] = v[q][0];
            El[1][i] = v[q][1];
            El[2][i] = v[q][2];
        }
    }
    __syncthreads();
    const float* lx = El[0];
    const float* ly = El[1];
    const float* lz = El[2];
    const int x = threadIdx.x % BT_X, y = threadIdx.x / BT_X;
    const int xw = t0[0] + x, yy = t0[1] + y;
    if (xw >= g.n[0] || yy >= g.n[1]) return;
    int xs = xw + origin;
    xs = xs >= g.n[0] ? xs - g.n[0] : xs;
#pragma unroll
    for (int zl = 0; zl < BT_Z; ++zl) {
        const int zz = t0[2] + zl;
        if (zz >= g.n[2]) break;
        const int o = ((zl + 1) * BS_Y + (y + 1)) * BS_X + (x + 1);
        const int idx = xs + g.n[0] * (yy + g.n[1] * zz);
        constexpr int X = 1, Y = BS_X, Z = BS_X * BS_Y;
        float dyEz = (sval_l<PD, 1>(c, lz, o + Y) - sval_l<PD, 1>(c, lz, o)) * g.inv_d[1];
        float dzEy = (sval_l<PD, 2>(c, ly, o + Z) - sval_l<PD, 2>(c, ly, o)) * g.inv_d[2];
        float dzEx = (sval_l<PD, 2>(c, lx, o + Z) - sval_l<PD, 2>(c, lx, o)) * g.inv_d[2];
        const float ezp = sval_l<PD, 0>(c, lz, o + X);
        const float eyp = sval_l<PD, 0>(c, ly, o + X);
        const float dxEz = (ezp - sval_l<PD, 0>(c, lz, o)) * g.inv_d[0];
        const float dxEy = (eyp - sval_l<PD, 0>(c, ly, o)) * g.inv_d[0];
        float dyEx = (sval_l<PD, 1>(c, lx, o + Y) - sval_l<PD, 1>(c, lx, o)) * g.inv_d[1];
        if (PML) {
            const int L2 = 2 * P.L;
            const int jl = pml_index(yy, g.n[1], P.L);
            if (jl >= 0) {
                const size_t q = (size_t)xs + (size_t)g.n[0] * (size_t)(jl + L2 * zz);
                const float b = P.coef[jl], bm1 = P.coef[L2 + jl];            // axis y, B kind
                dyEz = pml_stretch(P.y[0], q, b, bm1, dyEz, store);
                dyEx = pml_stretch(P.y[1], q, b, bm1, dyEx, store);
            }
            const int kl = pml_index(zz, g.n[2], P.L);
            if (kl >= 0) {
                const size_t q = (size_t)xs + (size_t)g.n[0] * (size_t)(yy + g.n[1] * kl);
                const float b = P.coef[4 * L2 + kl], bm1 = P.coef[5 * L2 + kl];  // axis z, B kind
                dzEy = pml_stretch(P.z[0], q, b, bm1, dzEy, store);
                dzEx = pml_stretch(P.z[1], q, b, bm1, dzEx, store);
            }
        }
        Bx[idx] -= h * (dyEz - dzEy);
        By[idx] -= h * (dzEx - dxEz);
        Bz[idx] -= h * (dxEy - dyEx);
    }
}

template <bool PD, bool PML>
__global__ void __launch_bounds__(BT_THREADS) k_bhalf_tiled(Geom g, PDCoef c, const float* __restrict__ Ex,
                                                           const float* __restrict__ Ey,
                                                           const float* __restrict__ Ez, float* __restrict__ Bx,
                                                           float* __restrict__ By, float* __restrict__ Bz, float h,
                                                           PmlDev P, int store) {
    __shared__ float El[3][BS_N];
    bhalf_tile<PD, PML>(g, c, Ex, Ey, Ez, Bx, By, Bz, h, blockIdx.x, blockIdx.y, blockIdx.z, El, P, store != 0);
}

// E += dt (curl B - J) with backward differences.
template <bool PML = false>
__device__ __forceinline__ void efull_cell(const Geom& g, float* __restrict__ Ex, float* __restrict__ Ey,
                                           float* __restrict__ Ez, const float* __restrict__ Bx,
                                           const float* __restrict__ By, const float* __restrict__ Bz,
                                           const float* __restrict__ Jx, const float* __restrict__ Jy,
                                           const float* __restrict__ Jz, int idx, const PmlDev* P = nullptr) {
    const Nbr n = neighbours(g, idx);
    const float bz = Bz[idx], by = By[idx], bx = Bx[idx];
    const float bzm_x = n.xm_ok ? Bz[at(g, n.im, n.j, n.k)] : 0.0f;
    const float bym_x = n.xm_ok ? By[at(g, n.im, n.j, n.k)] : 0.0f;
    const bool ym_ok = !PML || n.j > 0, zm_ok = !PML || n.k > 0;   // zero beyond the layer's outer faces
    float dyBz = (bz - (ym_ok ? Bz[at(g, n.i, n.jm, n.k)] : 0.0f)) * g.inv_d[1];
    float dzBy = (by - (zm_ok ? By[at(g, n.i, n.j, n.km)] : 0.0f)) * g.inv_d[2];
    float dzBx = (bx - (zm_ok ? Bx[at(g, n.i, n.j, n.km)] : 0.0f)) * g.inv_d[2];
    const float dxBz = (bz - bzm_x) * g.inv_d[0];
    const float dxBy = (by - bym_x) * g.inv_d[0];
    float dyBx = (bx - (ym_ok ? Bx[at(g, n.i, n.jm, n.k)] : 0.0f)) * g.inv_d[1];
    if (PML) {
        const int L2 = 2 * P->L;
        const int jl = pml_index(n.j, g.n[1], P->L);
        if (jl >= 0) {
            const size_t q = (size_t)n.i + (size_t)g.n[0] * (size_t)(jl + L2 * n.k);
            const float b = P->coef[2 * L2 + jl], bm1 = P->coef[3 * L2 + jl];   // axis y, E kind
            dyBz = pml_stretch(P->y[2], q, b, bm1, dyBz, true);
            dyBx = pml_stretch(P->y[3], q, b, bm1, dyBx, true);
        }
        const int kl = pml_index(n.k, g.n[2], P->L);
        if (kl >= 0) {
            const size_t q = (size_t)n.i + (size_t)g.n[0] * (size_t)(n.j + g.n[1] * kl);
            const float b = P->coef[6 * L2 + kl], bm1 = P->coef[7 * L2 + kl];   // axis z, E kind
            dzBy = pml_stretch(P->z[2], q, b, bm1, dzBy, true);
            dzBx = pml_stretch(P->z[3], q, b, bm1, dzBx, true);
        }
    }
    Ex[idx] += g.dt * ((dyBz - dzBy) - Jx[idx]);
    Ey[idx] += g.dt * ((dzBx - dxBz) - Jy[idx]);
    Ez[idx] += g.dt * ((dxBy - dyBx) - Jz[idx]);
}

template <bool PML>
__global__ void __launch_bounds__(256) k_efull(Geom g, float* __restrict__ Ex, float* __restrict__ Ey,
                                               float* __restrict__ Ez, const float* __restrict__ Bx,
                                               const float* __restrict__ By, const float* __restrict__ Bz,
                                               const float* __restrict__ Jx, const float* __restrict__ Jy,
                                               const float* __restrict__ Jz, PmlDev P) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ncell) return;
    efull_cell<PML>(g, Ex, Ey, Ez, Bx, By, Bz, Jx, Jy, Jz, idx, &P);
}

// Zero the layer's auxiliary values on storage x plane ix (the plane a
// window move turns into the new, empty leading plane).
__global__ void __launch_bounds__(256) k_clear_pml_plane(Geom g, PmlDev P, int ix) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int L2 = 2 * P.L;
    if (t < L2 * g.n[2]) {
        const int l = t % L2, k = t / L2;
        const size_t q = (size_t)ix + (size_t)g.n[0] * (size_t)(l + L2 * k);
#pragma unroll
        for (int a = 0; a < 4; ++a) P.y[a][q] = 0.0f;
    }
    if (t < g.n[1] * L2) {
        const int j = t % g.n[1], l = t / g.n[1];
        const size_t q = (size_t)ix + (size_t)g.n[0] * (size_t)(j + g.n[1] * l);
#pragma unroll
        for (int a = 0; a < 4; ++a) P.z[a][q] = 0.0f;
    }
}

// One (1/4, 1/2, 1/4) pass along each axis, as the separable 27-point product
// stencil, src -> dst (distinct buffers).
__device__ __forceinline__ void binomial_cell(const Geom& g, const float* __restrict__ s0,
                                              const float* __restrict__ s1, const float* __restrict__ s2,
                                              float* __restrict__ d0, float* __restrict__ d1,
                                              float* __restrict__ d2, int idx) {
    const Nbr n = neighbours(g, idx);
    const float wx[3] = {0.25f, 0.5f, 0.25f};
    const int xs[3] = {n.im, n.i, n.ip};
    const bool xok[3] = {n.xm_ok, true, n.xp_ok};
    const int ys[3] = {n.jm, n.j, n.jp};
    const int zs[3] = {n.km, n.k, n.kp};
    const float* src[3] = {s0, s1, s2};
    float* dst[3] = {d0, d1, d2};
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float ay = 0.0f;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                float ax = 0.0f;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (xok[a]) ax = fmaf(wx[a], src[comp][at(g, xs[a], ys[b], zs[c])], ax);
                ay = fmaf(wx[b], ax, ay);
            }
            acc = fmaf(wx[c], ay, acc);
        }
        dst[comp][idx] = acc;
    }
}

__global__ void __launch_bounds__(256) k_binomial(Geom g, const float* __restrict__ s0, const float* __restrict__ s1,
                                                  const float* __restrict__ s2, float* __restrict__ d0,
                                                  float* __restrict__ d1, float* __restrict__ d2) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ncell) return;
    binomial_cell(g, s0, s1, s2, d0, d1, d2, idx);
}

// Batched field kernels: grid y = member.
// Grid x = tile (x fastest) of the member's grid, y = member.
__global__ void __launch_bounds__(BT_THREADS) k_batch_bhalf(const InstDesc* __restrict__ tab) {
    __shared__ float El[3][BS_N];
    const InstDesc& d = tab[blockIdx.y];
    const Geom g = d.g;
    const int tx = (g.n[0] + BT_X - 1) / BT_X, ty = (g.n[1] + BT_Y - 1) / BT_Y, tz = (g.n[2] + BT_Z - 1) / BT_Z;
    const int t = blockIdx.x;
    if (t >= tx * ty * tz) return;
    const PDCoef c = d.c;
    const int bx = t % tx, by = (t / tx) % ty, bz = t / (tx * ty);
    const PmlDev none{};
    if (d.pd)
        bhalf_tile<true, false>(g, c, d.f.E[0], d.f.E[1], d.f.E[2], d.f.B[0], d.f.B[1], d.f.B[2], d.hdt, bx, by, bz,
                                El, none, false);
    else
        bhalf_tile<false, false>(g, c, d.f.E[0], d.f.E[1], d.f.E[2], d.f.B[0], d.f.B[1], d.f.B[2], d.hdt, bx, by, bz,
                                 El, none, false);
}

__global__ void __launch_bounds__(256) k_batch_efull(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.g.ncell) return;
    const Geom g = d.g;
    efull_cell(g, d.f.E[0], d.f.E[1], d.f.E[2], d.f.B[0], d.f.B[1], d.f.B[2], d.J[0], d.J[1], d.J[2], idx);
}

__global__ void __launch_bounds__(256) k_batch_binomial(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (!d.jpost || idx >= d.g.ncell) return;
    const Geom g = d.g;
    binomial_cell(g, d.Jt[0], d.Jt[1], d.Jt[2], d.J[0], d.J[1], d.J[2], idx);
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_bhalf(const Geom& g, int pd, const PDCoef& c, float* const E[3], float* const B[3], float h,
                        const PmlDev* pml, int store, hipStream_t st) {
    const dim3 nb((g.n[0] + BT_X - 1) / BT_X, (g.n[1] + BT_Y - 1) / BT_Y, (g.n[2] + BT_Z - 1) / BT_Z);
    const PmlDev P = pml ? *pml : PmlDev{};
    auto k = pd ? (pml ? k_bhalf_tiled<true, true> : k_bhalf_tiled<true, false>)
                : (pml ? k_bhalf_tiled<false, true> : k_bhalf_tiled<false, false>);
    hipLaunchKernelGGL(k, nb, dim3(BT_THREADS), 0, st, g, c, E[0], E[1], E[2], B[0], B[1], B[2], h, P, store);
    return hipGetLastError();
}

hipError_t launch_efull(const Geom& g, float* const E[3], float* const B[3], float* const J[3], const PmlDev* pml,
                        hipStream_t st) {
    const int nb = (g.ncell + 255) / 256;
    const PmlDev P = pml ? *pml : PmlDev{};
    hipLaunchKernelGGL(pml ? k_efull<true> : k_efull<false>, dim3(nb), dim3(256), 0, st, g, E[0], E[1], E[2], B[0],
                       B[1], B[2], J[0], J[1], J[2], P);
    return hipGetLastError();
}

hipError_t launch_clear_pml_plane(const Geom& g, const PmlDev& P, int ix, hipStream_t st) {
    const int n = std::max(2 * P.L * g.n[2], 2 * P.L * g.n[1]);
    hipLaunchKernelGGL(k_clear_pml_plane, dim3((n + 255) / 256), dim3(256), 0, st, g, P, ix);
    return hipGetLastError();
}

hipError_t launch_binomial(const Geom& g, float* const src[3], float* const dst[3], hipStream_t st) {
    const int nb = (g.ncell + 255) / 256;
    hipLaunchKernelGGL(k_binomial, dim3(nb), dim3(256), 0, st, g, src[0], src[1], src[2], dst[0], dst[1], dst[2]);
    return hipGetLastError();
}

hipError_t launch_batch_bhalf(const InstDesc* d, int n, int max_tiles, hipStream_t st) {
    if (n <= 0 || max_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_bhalf, dim3(max_tiles, n), dim3(BT_THREADS), 0, st, d);
    return hipGetLastError();
}

int bhalf_tiles(const int n[3]) {
    return ((n[0] + BT_X - 1) / BT_X) * ((n[1] + BT_Y - 1) / BT_Y) * ((n[2] + BT_Z - 1) / BT_Z);
}

hipError_t launch_batch_efull(const InstDesc* d, int n, int max_cells, hipStream_t st) {
    if (n <= 0 || max_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_efull, dim3((max_cells + 255) / 256, n), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_batch_binomial(const InstDesc* d, int n, int max_cells, hipStream_t st) {
    if (n <= 0 || max_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_binomial, dim3((max_cells + 255) / 256, n), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)nb), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace pic
