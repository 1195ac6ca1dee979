// Internal interface between the host ABI (pic_abi.hip) and the kernel
// translation units.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic_device.h"

namespace pic {

struct FieldPtrs {
    float* E[3];
    float* B[3];
};

// Transverse absorbing layer of L cells at each y and z edge: the auxiliary
// arrays of the convolutional form, each over the cells of its layer only,
// in storage x order (they move with the window like the fields).
//   y[0..3]: B_x by y, B_z by y, E_x by y, E_z by y; index i + nx (l + 2L k)
//   z[0..3]: B_x by z, B_y by z, E_x by z, E_y by z; index i + nx (j + ny l)
// l in [0, 2L) is the layer index of a cell: j for j < L, j - (n - 2L) for
// j >= n - L.  coef[((axis * 2 + kind) * 2 + which) * 2L + l]: axis 0 = y,
// 1 = z; kind 0 = the B updates (derivatives at l's half-integer position),
// 1 = the E update (integer position); which 0 = b = exp(-sigma dt),
// 1 = b - 1.
struct PmlDev {
    float* y[4];
    float* z[4];
    const float* coef;
    int L;
};

__host__ __device__ inline int pml_index(int j, int n, int L) {
    return j < L ? j : (j >= n - L ? j - (n - 2 * L) : -1);
}

// plasma profile (see pic_plasma_desc)
struct PlasmaDev {
    double x_start, ramp, n_plateau;
    int ppc[3];
};

// Division by a divisor d >= 1 fixed at set-up, for dividends n in [0, 2^31):
// floor(n / d) = (n m) >> s with s = 31 + ceil(log2 d) and m = ceil(2^s / d)
// < 2^33 (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Theorem 4.2: m d - 2^s < d <= 2^(s-31)).  A
// 32x64-bit multiply and a shift, where a general integer division takes some
// forty instructions.
struct FastDiv {
    unsigned long long m;
    int s;
};

inline FastDiv make_fastdiv(int d) {
    if (d < 1) return FastDiv{0ull, 0};   // (invalid sizes are rejected before any launch)
    int l = 0;
    while ((1ll << l) < (long long)d) ++l;
    FastDiv f;
    f.s = 31 + l;
    f.m = ((1ull << f.s) + (unsigned long long)d - 1ull) / (unsigned long long)d;
    return f;
}

__device__ __forceinline__ int fdiv(int n, const FastDiv& f) {
    return (int)(((unsigned long long)(unsigned)n * f.m) >> f.s);
}

// The divisors of the sort's key computation (cell -> coordinates -> tile).
struct SortDiv {
    FastDiv nx, nxy, T[3], tcells;
};

inline SortDiv make_sortdiv(const Geom& g, const TileGeom& t) {
    SortDiv d;
    d.nx = make_fastdiv(g.n[0]);
    d.nxy = make_fastdiv(g.nxy);
    for (int a = 0; a < 3; ++a) d.T[a] = make_fastdiv(t.T[a]);
    d.tcells = make_fastdiv(t.tcells);
    return d;
}

// One member of a batch of independent simulations for one species and one
// step, as the batched kernels see it (a device-resident table the host
// rewrites before each step).  Geometry is the one at the start of the step.
struct InstDesc {
    Geom g;
    TileGeom t;
    int guard;
    int pd;                  // perfect-dispersion smoothing in the B update
    int depth;               // in-tile order of the sort (0: levels, else the block-transpose depth)
    int nkeys;               // sort keys (t.ntiles * t.tcells)
    SortDiv sdiv;            // the sort's divisors for g and t
    PDCoef c;
    FieldPtrs f;
    float* J[3];             // current read by the E update
    float* Jt[3];            // workspace current (binomial filter source)
    int jpost;               // 0: none, 1: binomial filter
    int sorting;             // 1: sort s -> alt first (no copy pass: the tile step gathers from s); the step runs on alt
    SpeciesDev s;            // particle arrays at the start of the step
    SpeciesDev alt;          // the other array set
    int* hist;               // sort histogram, then its exclusive scan (member scratch)
    int* toff;               // tile ranges of the species (written by its sort)
    int* rank;
    int* sums;
    int* level;              // level-order places of a depth-0 sort (member scratch, max_particles ints)
    int* lc;                 // per-key local counts of a re-sort (member scratch, nkeys ints)
    int resort;              // 1: the sort's particles [0, *sorted) still sit in the tile ranges toff
    unsigned long long* acc;
    int* err;
    int* count;              // particles in the arrays
    int* sorted;             // particles inside the tile ranges of the last sort
    int* rest_n;             // entries on the species' rest list (the list is `rank`, idle between sorts)
    int capacity;
    float hdt;               // dt / 2
    double jscale[3];
    // laser source planes: B_z behind the source at t and t + dt, E_y on the
    // source at t + dt/2
    int laser_on;
    int lix_b, lix_e;
    double lcoef[3];
    double yc, zc, inv_w2, dy, dz;
    // moving window at the end of the step
    int wmove;               // 1: clear the plane at origin, origin += 1
    int inject;              // 1: load the species' plasma on window cell `slab` after the move
    int slab;
    long long shift;         // window shift after the move
    PlasmaDev plasma;
};

// Particles arrays the tile step of a batch member works on.
__host__ __device__ inline const SpeciesDev& step_arrays(const InstDesc& d) { return d.sorting ? d.alt : d.s; }

// batched kernels: one launch per phase over `n` members (grid y = member,
// except the tile step, whose work list is the concatenation of all tiles)
hipError_t launch_batch_sort(const InstDesc* d, int n, int max_particles, int max_keys1, int max_tiles1,
                             int max_tcells, hipStream_t st);
// all_888g1: every member tiles 8x8x8 with guard 1 (the compile-time tile body)
hipError_t launch_batch_tile(const InstDesc* d, const int* tile_begin, int n, int total_tiles, int threads,
                             size_t lds_bytes, bool all_888g1, hipStream_t st);
hipError_t launch_batch_rest(const InstDesc* d, int n, hipStream_t st);
hipError_t launch_batch_jfinal(const InstDesc* d, int n, int max_cells, hipStream_t st);
hipError_t launch_batch_binomial(const InstDesc* d, int n, int max_cells, hipStream_t st);
// B half step over the members' tiles (max_tiles = the largest bhalf_tiles of a member)
hipError_t launch_batch_bhalf(const InstDesc* d, int n, int max_tiles, hipStream_t st);
int bhalf_tiles(const int n[3]);
hipError_t launch_batch_efull(const InstDesc* d, int n, int max_cells, hipStream_t st);
// which: 0, 1, 2 = the laser planes in the order they are applied
hipError_t launch_batch_laser(const InstDesc* d, int n, int which, int max_plane, hipStream_t st);
hipError_t launch_batch_clear(const InstDesc* d, int n, int max_plane, hipStream_t st);
hipError_t launch_batch_inject(const InstDesc* d, int n, long long max_cand, hipStream_t st);

// Learned current denoiser (pic_denoise.hip): J' = B(J + sigma curl(net(J / s))).
// Packed bf16 weights:
// w1 [32 out][128] with k = tap * 4 + in (in < 3, tap < 27, else zero);
// w2 [27 tap][32 out][32 in]; w3 [27 tap][16 out][32 in] (out < 3, else zero);
// tap = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).  Biases FP32: b1[32], b2[32], b3[16].
struct DenoiseWeights {
    const __bf16* w1;
    const __bf16* w2;
    const __bf16* w3;
    const float* b1;
    const float* b2;
    const float* b3;
    float scale[3];
    float sigma;      // output stage J' = B(J + sigma curl(y)), sigma = dx (s_x + s_y + s_z) / 3
    float inv_d[3];
};
// bf16 elements; W3: 9 tap columns x 6 halo rows x 16 columns (4 row blocks x 4) x 32
constexpr size_t kDnW1 = 32 * 128, kDnW2 = 27 * 32 * 32, kDnW3 = 9 * 6 * 16 * 32;
constexpr size_t kDnBias = 32 + 32 + 16;                                            // floats

// bc per axis: 0 periodic, 1 zero outside the box, 2 moving window (zero
// beyond the window's ends).  Jin -> Jout (distinct), h1, h2: [ncell][32] bf16.
hipError_t launch_denoise(const Geom& g, const int bc[3], const DenoiseWeights& w, float* const Jin[3],
                          float* const Jout[3], __bf16* h1, __bf16* h2, hipStream_t st);

// window / injection / laser kernels (pic_window.hip)
hipError_t launch_clear_plane(const Geom& g, const FieldPtrs& f, int ix, hipStream_t st);
hipError_t launch_inject(const Geom& g, const PlasmaDev& P, const SpeciesDev& s, long long shift, int xb, int xe,
                         int* d_count, int capacity, int* d_err, hipStream_t st);
hipError_t launch_laser_plane(const Geom& g, float* F, int ix, double coef, double yc, double zc, double waist,
                              double dy, double dz, hipStream_t st);

// particle kernels (pic_particles.hip)
hipError_t launch_gather_push(const Geom& g, const FieldPtrs& f, const SpeciesDev& s, const PrevDev& prev,
                              const int* d_count, int max_count, int* d_err, hipStream_t st);
hipError_t launch_deposit(const Geom& g, const SpeciesDev& s, const PrevDev& prev, const int* d_count,
                          int max_count, unsigned long long* acc, hipStream_t st);
hipError_t launch_jfinal(const Geom& g, unsigned long long* acc, float* const J[3], const double scale[3],
                         int zero_acc, hipStream_t st);

// sort (pic_sort.hip): src -> dst, new count into d_count and d_sorted, tile
// ranges into toff (t.ntiles + 1 entries); hist, rank, sums are scratch.
// depth: 0 = level order inside a tile (level: scratch of max_count ints),
// else the in-tile block-transpose depth (1 = plain cell order; level
// unused).  copy = false leaves only each destination's source index in
// dst.cell: the next tile step (launch_pic_tile with src) then gathers the
// particles itself.  resort: particles [0, *d_sorted) still occupy the tile
// ranges toff of the last sort with this tiling (counted tile by tile; lc:
// scratch of t.ntiles * t.tcells ints).
hipError_t launch_sort(const Geom& g, const TileGeom& t, const SpeciesDev& src, const SpeciesDev& dst,
                       int* d_count, int* d_sorted, int max_count, int* hist, int* rank, int* sums, int* level,
                       int* lc, int depth, int* toff, bool copy, bool resort, hipStream_t st);

// fused tile kernel (pic_tile.hip)
size_t tile_lds_bytes(const TileGeom& t, int guard);
// toff: tile ranges of the species' last sort
// rest_n / rest_idx: the species' rest list (counter zeroed here, indices appended by the kernel)
// src: null, or the pre-sort arrays when the sort ran without its copy pass
// (s.cell then holds source indices; the step writes every array of s)
hipError_t launch_pic_tile(const Geom& g, const TileGeom& t, int guard, int threads, const FieldPtrs& f,
                           const SpeciesDev& s, const SpeciesDev* src, const int* toff, unsigned long long* acc,
                           int* d_err, int* rest_n, int* rest_idx, hipStream_t st);
// rest pass after the tile kernel: the particles on its rest list (beyond
// their tile's guard, marked cell -2 - c) and those appended after the last
// sort (index >= sorted)
hipError_t launch_tile_rest(const Geom& g, const FieldPtrs& f, const SpeciesDev& s, const int* d_sorted,
                            const int* d_count, const int* rest_n, const int* rest_idx, unsigned long long* acc,
                            int* d_err, hipStream_t st);

// field kernels (pic_fields.hip)
// pml: nullptr without the absorbing layer; store: the first of a step's two
// B half steps advances the layer's B arrays, the second only reads them.
hipError_t launch_bhalf(const Geom& g, int pd, const PDCoef& c, float* const E[3], float* const B[3], float h,
                        const PmlDev* pml, int store, hipStream_t st);
hipError_t launch_efull(const Geom& g, float* const E[3], float* const B[3], float* const J[3], const PmlDev* pml,
                        hipStream_t st);
hipError_t launch_clear_pml_plane(const Geom& g, const PmlDev& P, int ix, hipStream_t st);
hipError_t launch_binomial(const Geom& g, float* const src[3], float* const dst[3], hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st);

// reductions (pic_reduce.hip)
// out[0] += sum q w dV, out[1] += sum m w (gamma-1) dV (FP64); cnt[0] += live count
hipError_t launch_diag_particles(const Geom& g, const SpeciesDev& s, double q, double m, double dv,
                                 const int* d_count, int max_count, double* out, unsigned long long* cnt,
                                 hipStream_t st);
// out[2] += 1/2 sum (E^2 + B^2) dV; maxbits[0] = max |J| as float bits
hipError_t launch_diag_fields(const Geom& g, float* const E[3], float* const B[3], float* const J[3], double dv,
                              double* out, unsigned int* maxbits, hipStream_t st);
// rho += sign * q w S S S (FP64 atomics) for positions (cell, off)
hipError_t launch_rho(const Geom& g, const int* cell, float* const off[3], const float* w, double q, double sign,
                      const int* d_count, int max_count, double* rho, hipStream_t st);
// run diagnostics (pic_diag.hip)
int diag_max_bins();
hipError_t launch_axis_line(const Geom& g, const float* F, int j0, int k0, double ty, double tz, double* out,
                            hipStream_t st);
hipError_t launch_spectrum(const Geom& g, const SpeciesDev& s, const int* d_count, int max_count, int quantity,
                           double lo, double hi, int nbins, double qdv, double* charge, unsigned long long* count,
                           hipStream_t st);
hipError_t launch_beam_moments(const Geom& g, const SpeciesDev& s, const int* d_count, int max_count, double ux_min,
                               double dy, double dz, double* sums, hipStream_t st);
hipError_t launch_select(const Geom& g, const SpeciesDev& s, const int* d_count, int max_count, double ux_min,
                         int* ocell, float* ooff, float* oux, int* oid, int* counter, hipStream_t st);
hipError_t launch_field_moments(const Geom& g, float* const E[3], float* const B[3], int mask, double dx, double dv,
                                double* sums, hipStream_t st);

// Scratch of the allocation-free continuity check (pic_reduce.hip): the
// device address of this GPU's fixed scratch array (looked up once per
// device, with that device current).  Layout: NoAllocHead at offset 0, the
// FP64 charge density (at most kNoAllocMaxCells cells) at kNoAllocRhoOffset.
constexpr int kNoAllocMaxCells = 1 << 21;
constexpr size_t kNoAllocRhoOffset = 256;
struct NoAllocHead {
    double red[4];
    unsigned long long contmax;
    unsigned int jmax;
    unsigned int pad;
};
hipError_t noalloc_scratch(void** out);

// max over nodes of |rho dx/dt + sum_d (dx/d_d)(J_d - J_d[-e_d])| as double bits
// ry = dx/dy, rz = dx/dz
hipError_t launch_continuity(const Geom& g, const double* rho, float* const J[3], double dx_dt, double ry,
                             double rz, int filt, unsigned long long* maxbits, hipStream_t st);

}  // namespace pic
