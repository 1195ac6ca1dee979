// Laser-wakefield boundary kernels: clearing the plane that re-enters a moving
// window as its new leading plane, loading cold lattice plasma along a density
// ramp, and the total-field/scattered-field laser source corrections.
#include "pic_internal.h"
#include "pic_particle_ops.h"

namespace pic {

// Zero E and B on the storage plane x = ix.
__global__ void k_clear_plane(Geom g, FieldPtrs f, int ix) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.n[1] * g.n[2]) return;
    const int idx = ix + g.n[0] * t;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        f.E[c][idx] = 0.0f;
        f.B[c][idx] = 0.0f;
    }
}

// Lab-frame electron density (in n0) at x_cells (lab cells).
__device__ __forceinline__ double ramp_density(const PlasmaDev& P, double x) {
    if (x < P.x_start) return 0.0;
    if (P.ramp > 0.0 && x < P.x_start + P.ramp) return P.n_plateau * (x - P.x_start) / P.ramp;
    return P.n_plateau;
}

// One thread per (window cell in [xb, xe) x all y, z) x lattice slot.  Slots are
// claimed with one atomic per wavefront (ballot + prefix popcount).
__global__ void __launch_bounds__(256) k_inject(Geom g, PlasmaDev P, SpeciesDev s, long long shift, int xb, int xe,
                                                int* __restrict__ d_count, int capacity, int* __restrict__ d_err) {
    const int ppc = P.ppc[0] * P.ppc[1] * P.ppc[2];
    const long long ncand = (long long)(xe - xb) * g.n[1] * g.n[2] * ppc;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
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

// F[ix, j, k] += coef * exp(-((y_j - yc)^2 + (z_k - zc)^2) / waist^2) with
// y_j = (j + 1/2) dy, z_k = k dz (the E_y / B_z transverse positions).
__global__ void k_laser_plane(Geom g, float* __restrict__ F, int ix, double coef, double yc, double zc,
                              double inv_w2, double dy, double dz) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.n[1] * g.n[2]) return;
    const int j = t % g.n[1], k = t / g.n[1];
    const double y = (j + 0.5) * dy - yc, z = k * dz - zc;
    F[ix + g.n[0] * t] += (float)(coef * exp(-(y * y + z * z) * inv_w2));
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
