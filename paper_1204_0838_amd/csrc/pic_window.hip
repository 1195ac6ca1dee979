// Laser-wakefield boundary kernels: clearing the plane that re-enters a moving
// window as its new leading plane, loading cold lattice plasma along a density
// ramp, and the total-field/scattered-field laser source corrections.
#include "pic_internal.h"
#include "pic_particle_ops.h"

namespace pic {

// Zero E and B on the storage plane x = ix.
__device__ __forceinline__ void clear_one(const Geom& g, const FieldPtrs& f, int ix, int t) {
    const int idx = ix + g.n[0] * t;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        f.E[c][idx] = 0.0f;
        f.B[c][idx] = 0.0f;
    }
}

__global__ void k_clear_plane(Geom g, FieldPtrs f, int ix) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.n[1] * g.n[2]) return;
    clear_one(g, f, ix, t);
}

// Lab-frame electron density (in n0) at x_cells (lab cells).
__device__ __forceinline__ double ramp_density(const PlasmaDev& P, double x) {
    if (x < P.x_start) return 0.0;
    if (P.ramp > 0.0 && x < P.x_start + P.ramp) return P.n_plateau * (x - P.x_start) / P.ramp;
    return P.n_plateau;
}

// One thread per (window cell in [xb, xe) x all y, z) x lattice slot.  Slots are
// claimed with one atomic per wavefront (ballot + prefix popcount).  Every lane
// of a wavefront calls this (the ballot needs them all).
__device__ __forceinline__ void inject_one(const Geom& g, const PlasmaDev& P, const SpeciesDev& s, long long shift,
                                           int xb, int xe, int* __restrict__ d_count, int capacity,
                                           int* __restrict__ d_err, long long t) {
    const int ppc = P.ppc[0] * P.ppc[1] * P.ppc[2];
    const long long ncand = (long long)(xe - xb) * g.n[1] * g.n[2] * ppc;
    bool valid = false;
    int xw = 0, j = 0, k = 0, sl = 0;
    double ox = 0.0, oy = 0.0, oz = 0.0, n = 0.0;
    if (t < ncand) {
        // candidate order: x slowest, then y, z, lattice slot (matches the tag)
        sl = (int)(t % ppc);
        long long r = t / ppc;
        k = (int)(r % g.n[2]);
        r /= g.n[2];
        j = (int)(r % g.n[1]);
        xw = xb + (int)(r / g.n[1]);
        const int sx = sl % P.ppc[0], sy = (sl / P.ppc[0]) % P.ppc[1], sz = sl / (P.ppc[0] * P.ppc[1]);
        ox = (sx + 0.5) / P.ppc[0];
        oy = (sy + 0.5) / P.ppc[1];
        oz = (sz + 0.5) / P.ppc[2];
        n = ramp_density(P, (double)(shift + xw) + ox);
        valid = n > 0.0;
    }
    const unsigned long long ball = __ballot(valid);
    if (ball == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)ball) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(d_count, __popcll(ball));
    base = __shfl(base, leader, 64);
    if (!valid) return;
    const int slot = base + __popcll(ball & ((1ull << lane) - 1ull));
    if (slot >= capacity) {
        atomicOr(d_err, ERR_OVERFLOW);
        return;
    }
    int sx = xw + g.origin;
    if (sx >= g.n[0]) sx -= g.n[0];
    s.cell[slot] = sx + g.n[0] * (j + g.n[1] * k);
    s.off[0][slot] = (float)ox;
    s.off[1][slot] = (float)oy;
    s.off[2][slot] = (float)oz;
    s.u[0][slot] = 0.0f;
    s.u[1][slot] = 0.0f;
    s.u[2][slot] = 0.0f;
    s.w[slot] = (float)(n / ppc);
    const long long tag = (((shift + xw) * g.n[1] + j) * (long long)g.n[2] + k) * ppc + sl;
    s.id[slot] = (int)(tag & 0x7fffffffll);
}

__global__ void __launch_bounds__(256) k_inject(Geom g, PlasmaDev P, SpeciesDev s, long long shift, int xb, int xe,
                                                int* __restrict__ d_count, int capacity, int* __restrict__ d_err) {
    inject_one(g, P, s, shift, xb, xe, d_count, capacity, d_err, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// F[ix, j, k] += coef * exp(-((y_j - yc)^2 + (z_k - zc)^2) / waist^2) with
// y_j = (j + 1/2) dy, z_k = k dz (the E_y / B_z transverse positions).
__device__ __forceinline__ void laser_one(const Geom& g, float* __restrict__ F, int ix, double coef, double yc,
                                          double zc, double inv_w2, double dy, double dz, int t) {
    const int j = t % g.n[1], k = t / g.n[1];
    const double y = (j + 0.5) * dy - yc, z = k * dz - zc;
    F[ix + g.n[0] * t] += (float)(coef * exp(-(y * y + z * z) * inv_w2));
}

__global__ void k_laser_plane(Geom g, float* __restrict__ F, int ix, double coef, double yc, double zc,
                              double inv_w2, double dy, double dz) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.n[1] * g.n[2]) return;
    laser_one(g, F, ix, coef, yc, zc, inv_w2, dy, dz, t);
}

// Batched forms: grid y = member.
__global__ void __launch_bounds__(256) k_batch_laser(const InstDesc* __restrict__ tab, int which) {
    const InstDesc& d = tab[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const double coef = d.lcoef[which];
    if (!d.laser_on || t >= d.g.n[1] * d.g.n[2]) return;
    const Geom g = d.g;
    float* F = which == 1 ? d.f.E[1] : d.f.B[2];
    laser_one(g, F, which == 1 ? d.lix_e : d.lix_b, coef, d.yc, d.zc, d.inv_w2, d.dy, d.dz, t);
}

__global__ void __launch_bounds__(256) k_batch_clear(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!d.wmove || t >= d.g.n[1] * d.g.n[2]) return;
    const Geom g = d.g;
    const FieldPtrs f = d.f;
    clear_one(g, f, g.origin, t);
}

// Injection after the window moved: geometry with the advanced origin.
__global__ void __launch_bounds__(256) k_batch_inject(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    if (!d.inject) return;
    Geom g = d.g;
    if (d.wmove) g.origin = g.origin + 1 == g.n[0] ? 0 : g.origin + 1;
    const PlasmaDev P = d.plasma;
    const SpeciesDev s = step_arrays(d);
    inject_one(g, P, s, d.shift, d.slab, d.slab + 1, d.count, d.capacity, d.err,
               (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_batch_laser(const InstDesc* d, int n, int which, int max_plane, hipStream_t st) {
    if (n <= 0 || max_plane <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_laser, dim3((max_plane + 255) / 256, n), dim3(256), 0, st, d, which);
    return hipGetLastError();
}

hipError_t launch_batch_clear(const InstDesc* d, int n, int max_plane, hipStream_t st) {
    if (n <= 0 || max_plane <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_clear, dim3((max_plane + 255) / 256, n), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_batch_inject(const InstDesc* d, int n, long long max_cand, hipStream_t st) {
    if (n <= 0 || max_cand <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_inject, dim3((unsigned)((max_cand + 255) / 256), n), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_clear_plane(const Geom& g, const FieldPtrs& f, int ix, hipStream_t st) {
    const int n = g.n[1] * g.n[2];
    hipLaunchKernelGGL(k_clear_plane, dim3((n + 255) / 256), dim3(256), 0, st, g, f, ix);
    return hipGetLastError();
}

hipError_t launch_inject(const Geom& g, const PlasmaDev& P, const SpeciesDev& s, long long shift, int xb, int xe,
                         int* d_count, int capacity, int* d_err, hipStream_t st) {
    const long long ncand = (long long)(xe - xb) * g.n[1] * g.n[2] * P.ppc[0] * P.ppc[1] * P.ppc[2];
    if (ncand <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inject, dim3((unsigned)((ncand + 255) / 256)), dim3(256), 0, st, g, P, s, shift, xb, xe,
                       d_count, capacity, d_err);
    return hipGetLastError();
}

hipError_t launch_laser_plane(const Geom& g, float* F, int ix, double coef, double yc, double zc, double waist,
                              double dy, double dz, hipStream_t st) {
    const int n = g.n[1] * g.n[2];
    hipLaunchKernelGGL(k_laser_plane, dim3((n + 255) / 256), dim3(256), 0, st, g, F, ix, coef, yc, zc,
                       1.0 / (waist * waist), dy, dz);
    return hipGetLastError();
}

}  // namespace pic
