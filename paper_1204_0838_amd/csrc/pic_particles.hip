// Particle kernels of the split path: field gather + Boris push + move, and the
// charge-conserving cubic (Esirkepov) deposit into the fixed-point current.
#include "pic_internal.h"
#include "pic_particle_ops.h"

namespace pic {

__global__ void __launch_bounds__(256) k_gather_push(Geom g, FieldPtrs f, SpeciesDev s, PrevDev prev,
                                                     const int* __restrict__ d_count, int* __restrict__ d_err) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *d_count) return;
    int cell = s.cell[p];
    if (cell >= g.ncell) {   // invalid input: remove the particle rather than index outside the grid
        atomicOr(d_err, ERR_OVERFLOW);
        cell = -1;
        s.cell[p] = -1;
    }
    prev.cell[p] = cell;
    if (cell < 0) return;
    int c[3];
    decompose(g, cell, c);
    float off[3] = {s.off[0][p], s.off[1][p], s.off[2][p]};
#pragma unroll
    for (int d = 0; d < 3; ++d) prev.off[d][p] = off[d];
    if (particle_killed(g, c)) {
        s.cell[p] = -1;
        prev.cell[p] = -1;
        return;
    }
    GatherStencil st;
    gather_stencil(off, st);
    int ii[3][4], ih[3][4];
    const int stride[3] = {1, g.n[0], g.nxy};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            ii[d][a] = wrapi(c[d] - 1 + a, g.n[d]) * stride[d];
            ih[d][a] = wrapi(c[d] + st.hb[d] + a, g.n[d]) * stride[d];
        }
    float E[3], B[3];
    gather_fields(f.E, f.B, ii, ih, st, E, B);
    float u[3] = {s.u[0][p], s.u[1][p], s.u[2][p]};
    int flags = push_move(g, s.qmh, E, B, u, off, c);
    if (flags) atomicOr(d_err, flags);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s.u[d][p] = u[d];
        s.off[d][p] = off[d];
    }
    s.cell[p] = c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
}

// Emitter of deposit contributions into the global fixed-point accumulator.
struct GlobalEmit {
    unsigned long long* acc;
    int ncell;
    int X[5], Y[5], Z[5];
    __device__ __forceinline__ void add(int comp, int jx, int jy, int jz, long long k) const {
        atomicAdd(acc + ((size_t)comp * ncell + X[jx] + Y[jy] + Z[jz]), (unsigned long long)k);
    }
};

__global__ void __launch_bounds__(256) k_deposit(Geom g, SpeciesDev s, PrevDev prev,
                                                 const int* __restrict__ d_count,
                                                 unsigned long long* __restrict__ acc) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *d_count) return;
    const int cell1 = s.cell[p], cell0 = prev.cell[p];
    if ((unsigned)cell0 >= (unsigned)g.ncell || (unsigned)cell1 >= (unsigned)g.ncell) return;
    int c0[3], c1[3];
    decompose(g, cell0, c0);
    decompose(g, cell1, c1);
    const float o0[3] = {prev.off[0][p], prev.off[1][p], prev.off[2][p]};
    const float o1[3] = {s.off[0][p], s.off[1][p], s.off[2][p]};
    if (!moved(c0, c1, o0, o1)) return;
    Axis5 A[3];
    GlobalEmit em;
    em.acc = acc;
    em.ncell = g.ncell;
    const int stride[3] = {1, g.n[0], g.nxy};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int di = unwrap_shift(c1[d] - c0[d], g.n[d]);
        axis5(di, o0[d], o1[d], A[d]);
        int* dst = d == 0 ? em.X : (d == 1 ? em.Y : em.Z);
#pragma unroll
        for (int j = 0; j < 5; ++j) dst[j] = wrapi(c0[d] + A[d].base + j, g.n[d]) * stride[d];
    }
    esirkepov(A, s.mq * s.w[p], em);
}

__device__ __forceinline__ void jfinal_one(unsigned long long* __restrict__ acc, float* J0, float* J1, float* J2,
                                           int ncell, double s0, double s1, double s2, int zero_acc, int i) {
    const long long a0 = (long long)acc[i], a1 = (long long)acc[(size_t)ncell + i],
                    a2 = (long long)acc[2 * (size_t)ncell + i];
    J0[i] = (float)((double)a0 * s0);
    J1[i] = (float)((double)a1 * s1);
    J2[i] = (float)((double)a2 * s2);
    if (zero_acc) {
        acc[i] = 0ull;
        acc[(size_t)ncell + i] = 0ull;
        acc[2 * (size_t)ncell + i] = 0ull;
    }
}

__global__ void k_jfinal(unsigned long long* __restrict__ acc, float* J0, float* J1, float* J2, int ncell,
                         double s0, double s1, double s2, int zero_acc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncell) return;
    jfinal_one(acc, J0, J1, J2, ncell, s0, s1, s2, zero_acc, i);
}

// Batched read-out of the current (accumulator cleared); into the workspace
// current when the binomial filter follows.
__global__ void __launch_bounds__(256) k_batch_jfinal(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncell = d.g.ncell;
    if (i >= ncell) return;
    float* const* J = d.jpost ? d.Jt : d.J;
    jfinal_one(d.acc, J[0], J[1], J[2], ncell, d.jscale[0], d.jscale[1], d.jscale[2], 1, i);
}

hipError_t launch_batch_jfinal(const InstDesc* d, int n, int max_cells, hipStream_t st) {
    if (n <= 0 || max_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_jfinal, dim3((max_cells + 255) / 256, n), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_gather_push(const Geom& g, const FieldPtrs& f, const SpeciesDev& s, const PrevDev& prev,
                              const int* d_count, int max_count, int* d_err, hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    const int nb = (max_count + 255) / 256;
    hipLaunchKernelGGL(k_gather_push, dim3(nb), dim3(256), 0, st, g, f, s, prev, d_count, d_err);
    return hipGetLastError();
}

hipError_t launch_deposit(const Geom& g, const SpeciesDev& s, const PrevDev& prev, const int* d_count,
                          int max_count, unsigned long long* acc, hipStream_t st) {
    if (max_count <= 0) return hipSuccess;
    const int nb = (max_count + 255) / 256;
    hipLaunchKernelGGL(k_deposit, dim3(nb), dim3(256), 0, st, g, s, prev, d_count, acc);
    return hipGetLastError();
}

hipError_t launch_jfinal(const Geom& g, unsigned long long* acc, float* const J[3], const double scale[3],
                         int zero_acc, hipStream_t st) {
    const int nb = (g.ncell + 255) / 256;
    hipLaunchKernelGGL(k_jfinal, dim3(nb), dim3(256), 0, st, acc, J[0], J[1], J[2], g.ncell, scale[0], scale[1],
                       scale[2], zero_acc);
    return hipGetLastError();
}

}  // namespace pic
