// Run diagnostics of the kind Section 3.2 reports, computed on the device in
// FP64 from the live state: a field component along the laser axis (for the
// length of the accelerating phase), charge spectra in kinetic energy or u_x,
// beam moments for the normalised transverse emittance, the selection of
// accelerated particles with their tags (collection phase space), and the
// first moments of the electromagnetic energy along x (the laser centroid,
// Section 3.3).  Each kernel streams its inputs once; sums use FP64 atomics
// after a wavefront reduction (histograms: per-workgroup LDS bins first).
#include "pic_internal.h"
#include "pic_particle_ops.h"

namespace pic {

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Window x index of storage x index i.
__device__ __forceinline__ int window_x(const Geom& g, int i) {
    if (!g.window) return i;
    const int xw = i - g.origin;
    return xw < 0 ? xw + g.n[0] : xw;
}

// A live particle: valid cell, not in a window kill zone or the transverse
// absorbing layer (removed at the next step).
__device__ __forceinline__ bool live_cell(const Geom& g, int cl) {
    if ((unsigned)cl >= (unsigned)g.ncell) return false;
    int c[3];
    decompose(g, cl, c);
    return !particle_killed(g, c);
}

__global__ void __launch_bounds__(256) k_axis_line(Geom g, const float* __restrict__ F, int j0, int k0, double ty,
                                                   double tz, double* __restrict__ out) {
    const int xw = blockIdx.x * blockDim.x + threadIdx.x;
    if (xw >= g.n[0]) return;
    int i = xw;
    if (g.window) {
        i = xw + g.origin;
        if (i >= g.n[0]) i -= g.n[0];
    }
    const int ja = j0 % g.n[1], jb = (j0 + 1) % g.n[1];
    const int ka = k0 % g.n[2], kb = (k0 + 1) % g.n[2];
    double acc = 0.0;
    acc += ((1.0 - tz) * (1.0 - ty)) * (double)F[i + g.n[0] * (ja + g.n[1] * ka)];
    acc += ((1.0 - tz) * ty) * (double)F[i + g.n[0] * (jb + g.n[1] * ka)];
    acc += (tz * (1.0 - ty)) * (double)F[i + g.n[0] * (ja + g.n[1] * kb)];
    acc += (tz * ty) * (double)F[i + g.n[0] * (jb + g.n[1] * kb)];
    out[xw] = acc;
}

constexpr int kMaxBins = 2048;

__global__ void __launch_bounds__(256) k_spectrum(Geom g, SpeciesDev s, const int* __restrict__ d_count, int quantity,
                                                  double lo, double hi, int nbins, double qdv,
                                                  double* __restrict__ charge, unsigned long long* __restrict__ count) {
    __shared__ double hq[kMaxBins];
    __shared__ unsigned long long hc[kMaxBins];
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        hq[b] = 0.0;
        hc[b] = 0ull;
    }
    __syncthreads();
    const int n = *d_count;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        if (!live_cell(g, s.cell[p])) continue;
        const double a = s.u[0][p];
        double val;
        if (quantity == 0) {
            const double b = s.u[1][p], c = s.u[2][p];
            const double u2 = a * a + b * b + c * c;
            val = u2 / (sqrt(1.0 + u2) + 1.0);   // gamma - 1 without cancellation
        } else {
            val = a;
        }
        const double t = (val - lo) / (hi - lo) * (double)nbins;
        const double idx = floor(t);
        if (!(t >= 0.0) || !(idx < (double)nbins)) continue;
        const int k = (int)idx;
        atomicAdd(&hq[k], qdv * (double)s.w[p]);
        atomicAdd(&hc[k], 1ull);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        if (hc[b]) {
            atomicAdd(charge + b, hq[b]);
            atomicAdd(count + b, hc[b]);
        }
    }
}

// sums: [0] w, [1] w u_x, then for y (2..6) and z (7..11): w r, w r^2, w p, w p^2, w p r; [12] count
__global__ void __launch_bounds__(256) k_beam_moments(Geom g, SpeciesDev s, const int* __restrict__ d_count,
                                                      double ux_min, double dy, double dz, double* __restrict__ sums) {
    double acc[13];
#pragma unroll
    for (int k = 0; k < 13; ++k) acc[k] = 0.0;
    const int n = *d_count;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const int cl = s.cell[p];
        if (!live_cell(g, cl)) continue;
        const double ux = s.u[0][p];
        if (!(ux > ux_min)) continue;
        const int j = (cl / g.n[0]) % g.n[1], k = cl / g.nxy;
        const double w = s.w[p];
        const double r[2] = {((double)j + (double)s.off[1][p]) * dy, ((double)k + (double)s.off[2][p]) * dz};
        const double pm[2] = {s.u[1][p], s.u[2][p]};
        acc[0] += w;
        acc[1] += w * ux;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            acc[2 + 5 * a] += w * r[a];
            acc[3 + 5 * a] += w * (r[a] * r[a]);
            acc[4 + 5 * a] += w * pm[a];
            acc[5 + 5 * a] += w * (pm[a] * pm[a]);
            acc[6 + 5 * a] += w * (pm[a] * r[a]);
        }
        acc[12] += 1.0;
    }
#pragma unroll
    for (int k = 0; k < 13; ++k) {
        const double v = wsum(acc[k]);
        if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(sums + k, v);
    }
}

// Compaction of the particles with u_x > ux_min: their cell, x offset, u_x
// and tag, at slots reserved with one atomic per wavefront.
__global__ void __launch_bounds__(256) k_select(Geom g, SpeciesDev s, const int* __restrict__ d_count, double ux_min,
                                                int* __restrict__ ocell, float* __restrict__ ooff,
                                                float* __restrict__ oux, int* __restrict__ oid,
                                                int* __restrict__ counter) {
    const int n = *d_count;
    const int lane = threadIdx.x & 63;
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int p = base + threadIdx.x;
        bool take = false;
        if (p < n) {
            const int cl = s.cell[p];
            take = live_cell(g, cl) && (double)s.u[0][p] > ux_min;
        }
        const unsigned long long m = __ballot(take);
        if (m == 0ull) continue;
        int slot0 = 0;
        if (lane == 0) slot0 = atomicAdd(counter, __popcll(m));
        slot0 = __shfl(slot0, 0, 64);
        if (take) {
            const int at = slot0 + __popcll(m & ((1ull << lane) - 1ull));
            ocell[at] = s.cell[p];
            ooff[at] = s.off[0][p];
            oux[at] = s.u[0][p];
            oid[at] = s.id[p];
        }
    }
}

// sums: [0] e dV, [1] e x dV, [2] e x^2 dV, e = F^2 / 2 of each used component
__global__ void __launch_bounds__(256) k_field_moments(Geom g, const float* __restrict__ F0,
                                                       const float* __restrict__ F1, const float* __restrict__ F2,
                                                       const float* __restrict__ F3, const float* __restrict__ F4,
                                                       const float* __restrict__ F5, int mask, double dx, double dv,
                                                       double* __restrict__ sums) {
    const float* F[6] = {F0, F1, F2, F3, F4, F5};
    const double stag[6] = {0.5, 0.0, 0.0, 0.0, 0.5, 0.5};
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.ncell; idx += gridDim.x * blockDim.x) {
        const int xw = window_x(g, idx % g.n[0]);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            if (!(mask & (1 << c))) continue;
            const double v = F[c][idx];
            const double e = 0.5 * (v * v) * dv;
            const double x = ((double)xw + stag[c]) * dx;
            m0 += e;
            m1 += e * x;
            m2 += e * x * x;
        }
    }
    m0 = wsum(m0);
    m1 = wsum(m1);
    m2 = wsum(m2);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(sums + 0, m0);
        atomicAdd(sums + 1, m1);
        atomicAdd(sums + 2, m2);
    }
}

int grid_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int diag_max_bins() { return kMaxBins; }

hipError_t launch_axis_line(const Geom& g, const float* F, int j0, int k0, double ty, double tz, double* out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_axis_line, dim3((g.n[0] + 255) / 256), dim3(256), 0, st, g, F, j0, k0, ty, tz, out);
    return hipGetLastError();
}

hipError_t launch_spectrum(const Geom& g, const SpeciesDev& s, const int* d_count, int max_count, int quantity,
                           double lo, double hi, int nbins, double qdv, double* charge, unsigned long long* count,
                           hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spectrum, dim3(grid_of(max_count)), dim3(256), 0, st, g, s, d_count, quantity, lo, hi, nbins,
                       qdv, charge, count);
    return hipGetLastError();
}

hipError_t launch_beam_moments(const Geom& g, const SpeciesDev& s, const int* d_count, int max_count, double ux_min,
                               double dy, double dz, double* sums, hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_beam_moments, dim3(grid_of(max_count)), dim3(256), 0, st, g, s, d_count, ux_min, dy, dz,
                       sums);
    return hipGetLastError();
}

hipError_t launch_select(const Geom& g, const SpeciesDev& s, const int* d_count, int max_count, double ux_min,
                         int* ocell, float* ooff, float* oux, int* oid, int* counter, hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3(grid_of(max_count)), dim3(256), 0, st, g, s, d_count, ux_min, ocell, ooff, oux,
                       oid, counter);
    return hipGetLastError();
}

hipError_t launch_field_moments(const Geom& g, float* const E[3], float* const B[3], int mask, double dx, double dv,
                                double* sums, hipStream_t st) {
    hipLaunchKernelGGL(k_field_moments, dim3(grid_of(g.ncell)), dim3(256), 0, st, g, E[0], E[1], E[2], B[0], B[1],
                       B[2], mask, dx, dv, sums);
    return hipGetLastError();
}

}  // namespace pic
