// FP64 global reductions: charge, kinetic and field energy, max |J|, and the
// continuity residual of the last deposit (rho re-deposited in FP64 from the
// stored FP32 positions).
#include <mutex>

#include "pic_internal.h"
#include "pic_particle_ops.h"

namespace pic {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_maxd(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ void __launch_bounds__(256) k_diag_particles(Geom g, const int* __restrict__ cell, const float* __restrict__ ux,
                                                        const float* __restrict__ uy, const float* __restrict__ uz,
                                                        const float* __restrict__ w, const int* __restrict__ d_count,
                                                        double qdv, double mdv, double* out,
                                                        unsigned long long* cnt) {
    const int n = *d_count;
    double q = 0.0, k = 0.0;
    unsigned long long live = 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const int cl = cell[p];
        if ((unsigned)cl >= (unsigned)g.ncell) continue;
        int cc[3];
        decompose(g, cl, cc);
        if (particle_killed(g, cc)) continue;   // removed at the next step
        const double a = ux[p], b = uy[p], c = uz[p];
        const double u2 = a * a + b * b + c * c;
        q += qdv * (double)w[p];
        // gamma - 1 = u^2 / (gamma + 1) avoids cancellation for slow particles
        k += mdv * (double)w[p] * (u2 / (sqrt(1.0 + u2) + 1.0));
        ++live;
    }
    q = wave_sum(q);
    k = wave_sum(k);
    for (int o = 32; o > 0; o >>= 1) live += __shfl_xor(live, o, 64);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out + 0, q);
        atomicAdd(out + 1, k);
        atomicAdd(cnt, live);
    }
}

__global__ void __launch_bounds__(256) k_diag_fields(int ncell, const float* __restrict__ E0,
                                                     const float* __restrict__ E1, const float* __restrict__ E2,
                                                     const float* __restrict__ B0, const float* __restrict__ B1,
                                                     const float* __restrict__ B2, const float* __restrict__ J0,
                                                     const float* __restrict__ J1, const float* __restrict__ J2,
                                                     double hdv, double* out, unsigned int* maxbits) {
    double e = 0.0;
    float mj = 0.0f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x) {
        const double a0 = E0[i], a1 = E1[i], a2 = E2[i], b0 = B0[i], b1 = B1[i], b2 = B2[i];
        e += a0 * a0 + a1 * a1 + a2 * a2 + b0 * b0 + b1 * b1 + b2 * b2;
        mj = fmaxf(mj, fmaxf(fabsf(J0[i]), fmaxf(fabsf(J1[i]), fabsf(J2[i]))));
    }
    e = wave_sum(e);
    mj = wave_maxf(mj);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out + 2, e * hdv);
        atomicMax(maxbits, __float_as_uint(mj));   // non-negative floats order like their bits
    }
}

__global__ void __launch_bounds__(256) k_rho(Geom g, const int* __restrict__ cell, const float* __restrict__ ox,
                                             const float* __restrict__ oy, const float* __restrict__ oz,
                                             const float* __restrict__ w, const int* __restrict__ d_count,
                                             double qs, double* __restrict__ rho) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *d_count) return;
    const int cl = cell[p];
    if ((unsigned)cl >= (unsigned)g.ncell) return;
    int c[3];
    decompose(g, cl, c);
    const double off[3] = {ox[p], oy[p], oz[p]};
    double wt[3][4];
    int ix[3][4];
    const int stride[3] = {1, g.n[0], g.nxy};
    for (int d = 0; d < 3; ++d) {
        const double t = off[d], t2 = t * t, t3 = t2 * t, e = 1.0 - t;
        wt[d][0] = e * e * e / 6.0;
        wt[d][1] = 2.0 / 3.0 - t2 + 0.5 * t3;
        wt[d][2] = (1.0 + 3.0 * t + 3.0 * t2 - 3.0 * t3) / 6.0;
        wt[d][3] = t3 / 6.0;
        for (int a = 0; a < 4; ++a) ix[d][a] = wrapi(c[d] - 1 + a, g.n[d]) * stride[d];
    }
    const double qw = qs * (double)w[p];
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i)
                atomicAdd(rho + (ix[0][i] + ix[1][j] + ix[2][k]), qw * wt[0][i] * wt[1][j] * wt[2][k]);
}

// filt: the current was post-processed by the binomial filter B (alone, or
// as the last stage of the denoiser's J' = B(J + sigma curl y), whose
// divergence is B div J): the charge is then B rho, evaluated here as the
// same 27-point product stencil (zero across the window seam, periodic y and
// z; the layer's cells hold no charge).
__global__ void __launch_bounds__(256) k_continuity(Geom g, const double* __restrict__ rho,
                                                    const float* __restrict__ J0, const float* __restrict__ J1,
                                                    const float* __restrict__ J2, double dx_dt, double ry,
                                                    double rz, int filt, unsigned long long* maxbits) {
    double m = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.ncell; idx += gridDim.x * blockDim.x) {
        const int k = idx / g.nxy;
        const int r = idx - k * g.nxy;
        const int j = r / g.n[0];
        const int i = r - j * g.n[0];
        const int im = i == 0 ? g.n[0] - 1 : i - 1;
        const int jm = j == 0 ? g.n[1] - 1 : j - 1;
        const int km = k == 0 ? g.n[2] - 1 : k - 1;
        bool xm_ok = true, xp_ok = true;
        if (g.window) {
            int xw = i - g.origin;
            if (xw < 0) xw += g.n[0];
            xm_ok = xw != 0;
            xp_ok = xw != g.n[0] - 1;
        }
        double q = rho[idx];
        if (filt) {
            const int ip = i + 1 == g.n[0] ? 0 : i + 1;
            const int jp = j + 1 == g.n[1] ? 0 : j + 1;
            const int kp = k + 1 == g.n[2] ? 0 : k + 1;
            const int xs[3] = {im, i, ip}, ys[3] = {jm, j, jp}, zs[3] = {km, k, kp};
            const bool xok[3] = {xm_ok, true, xp_ok};
            const double wt[3] = {0.25, 0.5, 0.25};
            q = 0.0;
            for (int c = 0; c < 3; ++c)
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a)
                        if (xok[a]) q += wt[a] * wt[b] * wt[c] * rho[xs[a] + g.n[0] * (ys[b] + g.n[1] * zs[c])];
        }
        const double jxm = xm_ok ? (double)J0[im + g.n[0] * (j + g.n[1] * k)] : 0.0;
        double res = q * dx_dt + ((double)J0[idx] - jxm);
        res += ry * ((double)J1[idx] - (double)J1[i + g.n[0] * (jm + g.n[1] * k)]);
        res += rz * ((double)J2[idx] - (double)J2[i + g.n[0] * (j + g.n[1] * km)]);
        m = fmax(m, fabs(res));
    }
    m = wave_maxd(m);
    if ((threadIdx.x & 63) == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
}

static int grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_diag_particles(const Geom& g, const SpeciesDev& s, double q, double m, double dv,
                                 const int* d_count, int max_count, double* out, unsigned long long* cnt,
                                 hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag_particles, dim3(grid_for(max_count)), dim3(256), 0, st, g, s.cell, s.u[0], s.u[1], s.u[2],
                       s.w, d_count, q * dv, m * dv, out, cnt);
    return hipGetLastError();
}

hipError_t launch_diag_fields(const Geom& g, float* const E[3], float* const B[3], float* const J[3], double dv,
                              double* out, unsigned int* maxbits, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_fields, dim3(grid_for(g.ncell)), dim3(256), 0, st, g.ncell, E[0], E[1], E[2], B[0],
                       B[1], B[2], J[0], J[1], J[2], 0.5 * dv, out, maxbits);
    return hipGetLastError();
}

hipError_t launch_rho(const Geom& g, const int* cell, float* const off[3], const float* w, double q, double sign,
                      const int* d_count, int max_count, double* rho, hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rho, dim3((max_count + 255) / 256), dim3(256), 0, st, g, cell, off[0], off[1], off[2], w,
                       d_count, q * sign, rho);
    return hipGetLastError();
}

hipError_t launch_continuity(const Geom& g, const double* rho, float* const J[3], double dx_dt, double ry,
                             double rz, int filt, unsigned long long* maxbits, hipStream_t st) {
    hipLaunchKernelGGL(k_continuity, dim3(grid_for(g.ncell)), dim3(256), 0, st, g, rho, J[0], J[1], J[2], dx_dt, ry,
                       rz, filt, maxbits);
    return hipGetLastError();
}

// ---- allocation-free continuity check --------------------------------------
// The scratch of pic_continuity_noalloc: a fixed device array (one per GPU,
// held until the process ends) instead of the caller's workspace.  Words
// 0..31 hold the reduction results (see NoAllocHead), the FP64 charge
// density follows at kNoAllocRhoOffset.
static __device__ __align__(256) unsigned char scratch[kNoAllocRhoOffset + (size_t)kNoAllocMaxCells * 8];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

hipError_t noalloc_scratch(void** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace pic
