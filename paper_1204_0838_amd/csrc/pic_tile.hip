// Fused gather + push + move + deposit over cell-sorted particle tiles.
//
// One workgroup per tile of T[0] x T[1] x T[2] cells.  The workgroup stages
// E and B of the tile plus a halo of H = guard + 2 cells in LDS, zeroes an
// int64 current tile covering the tile plus guard + 2 (low) / guard + 3 (high)
// cells, and then streams its particles (coalesced SoA loads):
//   particles still within `guard` cells of the tile: gather from LDS,
//     deposit with LDS 64-bit atomics;
//   particles that drifted further since the last sort: left for a second
//     kernel (their cell index is replaced by -2 - cell and their index is
//     appended to the species' rest list, one atomic per wavefront), which
//     gathers from global memory and deposits with global atomics (the same
//     arithmetic).  Keeping that path out of the tile kernel keeps its loop
//     free of calls, so the kernel arguments stay in scalar registers.
// Finally the non-zero LDS current is added to the global fixed-point
// accumulator in one atomic pass.  The step right after a sort also does the
// sort's gather: the sort leaves each destination's source index in the
// cell array, and this kernel reads every particle through it from the
// pre-sort arrays and writes all of its arrays at the destination.  Every value goes through the same device
// functions as the split kernels, so the fused and split paths agree bit for
// bit (integer sums are order-independent).
//
// Workgroups are mapped to tiles XCD by XCD: consecutive workgroup indices go
// round-robin over the 8 XCDs, and the tiles are dealt to the XCDs in chunks
// (a row of tiles along x for one grid, 8 tiles of the concatenated list for a
// batch): XCD k takes chunks k, k + 8, k + 16, ...  Neighbouring tiles of a
// row share their halos in that XCD's L2, while a dense region (the wake on
// the axis) is spread over all XCDs instead of loading one of them.
#include <algorithm>

#include "pic_internal.h"
#include "pic_particle_ops.h"

namespace pic {

// LDS current tile, addressed by slots relative to the particle's old cell
// (esirkepov<true>): `base` is the lane's node at its old cell - 1 along each
// axis (slot 0, component 0), and every core slot is base plus an offset
// that is a compile-time constant for the compiled tile shapes (the whole
// core stencil of all three components lies within the 16-bit immediate
// offset of ds_add_u64), so lanes in distinct cells stay in distinct banks
// whether or not, and which way, they crossed a cell face.  Only the one
// extra slot of a crossing axis takes a per-lane correction: it is written
// as the forward node (slot 4 = old cell + 3, or along the component's own
// axis slot 3 = old cell + 2) and moved to old cell - 2 for a backward
// crossing.
struct LdsEmit {
    unsigned long long* base;
    int jx, jpl, jr;                // row, plane and component strides
    int dxm, dym, dzm;              // backward corrections of the transverse extra slot (elements)
    int dxp, dyp, dzp;              // ... and of the own-axis extra slot
    __device__ __forceinline__ void add(int comp, int sx, int sy, int sz, long long k) const {
        const int off = comp * jr + sx + sy * jx + sz * jpl;
        int corr = 0;
        if (comp == 0 ? sx == 3 : sx == 4) corr += comp == 0 ? dxp : dxm;
        if (comp == 1 ? sy == 3 : sy == 4) corr += comp == 1 ? dyp : dym;
        if (comp == 2 ? sz == 3 : sz == 4) corr += comp == 2 ? dzp : dzm;
        atomicAdd(base + (off + corr), (unsigned long long)k);
    }
};

struct GlobalEmitT {
    unsigned long long* acc;
    int ncell;
    int X[5], Y[5], Z[5];
    __device__ __forceinline__ void add(int comp, int jx, int jy, int jz, long long k) const {
        atomicAdd(acc + ((size_t)comp * ncell + X[jx] + Y[jy] + Z[jz]), (unsigned long long)k);
    }
};

// Tile of workgroup b when chunks of `chunk` consecutive tiles are dealt
// round-robin to the 8 XCDs (>= ntiles: no tile; grid = xcd_blocks).
// v mod n in [0, n) for any v; a single compare when v is already inside
// (the staging and flush loops wrap only at the domain's faces).
__device__ __forceinline__ int wrap_any(int v, int n) {
    return (unsigned)v < (unsigned)n ? v : ((v % n) + n) % n;
}

__device__ __forceinline__ int xcd_tile(int b, int ntiles, int chunk) {
    const int k = b % 8, j = b / 8;
    const int c = k + 8 * (j / chunk);
    const long long tile = (long long)c * chunk + j % chunk;
    return tile < ntiles ? (int)tile : ntiles;
}

static int xcd_blocks(int ntiles, int chunk) {
    const int nchunks = (ntiles + chunk - 1) / chunk;
    return 8 * ((nchunks + 7) / 8) * chunk;
}

constexpr int kBatchChunk = 8;

// One particle (index p, cell coordinates c) through global memory: gather,
// push, move, store, deposit with global atomics.  Returns error flags.
__device__ __forceinline__ int push_deposit_global(const Geom& g, const FieldPtrs& f, const SpeciesDev& s, int p,
                                                const int c[3], unsigned long long* acc) {
    const int gstride[3] = {1, g.n[0], g.nxy};
    float o[3] = {s.off[0][p], s.off[1][p], s.off[2][p]};
    const float o0[3] = {o[0], o[1], o[2]};
    float u[3] = {s.u[0][p], s.u[1][p], s.u[2][p]};
    GatherStencil st;
    gather_stencil(o, st);
    int ii[3][4], ih[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            ii[d][a] = wrapi(c[d] - 1 + a, g.n[d]) * gstride[d];
            ih[d][a] = wrapi(c[d] + st.hb[d] + a, g.n[d]) * gstride[d];
        }
    float E[3], B[3];
    gather_fields(f.E, f.B, ii, ih, st, E, B);
    int c1[3] = {c[0], c[1], c[2]};
    const int errs = push_move(g, s.qmh, E, B, u, o, c1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s.u[d][p] = u[d];
        s.off[d][p] = o[d];
    }
    s.cell[p] = c1[0] + g.n[0] * (c1[1] + g.n[1] * c1[2]);
    if (!moved(c, c1, o0, o)) return errs;
    Axis5 A[3];
    GlobalEmitT em;
    em.acc = acc;
    em.ncell = g.ncell;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        axis5(unwrap_shift(c1[d] - c[d], g.n[d]), o0[d], o[d], A[d]);
        int* dst = d == 0 ? em.X : (d == 1 ? em.Y : em.Z);
#pragma unroll
        for (int j = 0; j < 5; ++j) dst[j] = wrapi(c[d] + A[d].base + j, g.n[d]) * gstride[d];
    }
    esirkepov(A, s.mq * s.w[p], em);
    return errs;
}

// Plane (z) strides of the two LDS regions, padded so that one z step moves
// the address by 8 banks: fields in 4-byte words mod 32, current in 8-byte
// words mod 16.  The sort stores a tile's cells as 8x2x4 bricks (x, then 4 z,
// then 2 y), so at 8 particles per cell the lanes of one LDS pass (32 for
// the b32 field reads, 16 for the int64 atomics) sit in 8 x-cells of 4 (or
// 2) successive z-planes and address disjoint banks.
__host__ __device__ constexpr int pad_plane(int p, int m) { return p + ((8 - p % m) + m) % m; }
__host__ __device__ constexpr int field_plane(int fx, int fy) { return pad_plane(fx * fy, 32); }
__host__ __device__ constexpr int cur_plane(int jx, int jy) { return pad_plane(jx * jy, 16); }

// Load particle pn of the tile's range.  With GATHER the step runs right
// after a sort that left only each destination's source index in s.cell:
// the particle is read from src at that index, and w and id, which the step
// does not change, are written to the destination at once (the step writes
// the other arrays), so the sort needs no copy pass of its own.
template <bool GATHER>
__device__ __forceinline__ void load_particle(const SpeciesDev& s, const SpeciesDev& src, int pn, int& cell,
                                              float o[3], float u[3], float& w) {
    if (GATHER) {
        const int ps = s.cell[pn];
        cell = src.cell[ps];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            o[d] = src.off[d][ps];
            u[d] = src.u[d][ps];
        }
        w = src.w[ps];
        s.w[pn] = w;
        s.id[pn] = src.id[ps];
    } else {
        cell = s.cell[pn];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            o[d] = s.off[d][pn];
            u[d] = s.u[d][pn];
        }
        w = s.w[pn];
    }
}

// Offsets and momenta of particle p written unchanged (a gathering step's
// particles that it does not push here still need them at their new place).
template <bool GATHER>
__device__ __forceinline__ void keep_particle(const SpeciesDev& s, int p, const float o[3], const float u[3]) {
    if (GATHER) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            s.off[d][p] = o[d];
            s.u[d][p] = u[d];
        }
    }
}

// Body of the fused step for one tile (the whole workgroup cooperates).
// TX, TY, TZ > 0 and GD >= 0 fix the tile shape and guard at compile time:
// every LDS stride is then a constant and each particle's current atomics
// and field reads address LDS as one base register plus immediate offsets.
// 0 (-1 for GD) takes them from t and guard_rt.
template <int NT, int TX = 0, int TY = 0, int TZ = 0, int GD = -1, bool GATHER = false>
__device__ __forceinline__ void tile_body(const Geom& g, const TileGeom& t, int guard_rt, const FieldPtrs& f,
                                          const SpeciesDev& s, const SpeciesDev& src, const int* __restrict__ toff,
                                          unsigned long long* __restrict__ acc, int* __restrict__ d_err,
                                          int* __restrict__ rest_n, int* __restrict__ rest_idx,
                                          unsigned long long* lds_u64, int tile) {
    const int T[3] = {TX > 0 ? TX : t.T[0], TY > 0 ? TY : t.T[1], TZ > 0 ? TZ : t.T[2]};
    const int guard = GD >= 0 ? GD : guard_rt;
    const int tz = tile / (t.nt[0] * t.nt[1]);
    const int tr = tile - tz * t.nt[0] * t.nt[1];
    const int ty = tr / t.nt[0];
    const int tx = tr - ty * t.nt[0];
    const int t0[3] = {tx * T[0], ty * T[1], tz * T[2]};
    int te[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) te[d] = min(T[d], g.n[d] - t0[d]);
    const int H = guard + 2;
    // LDS geometry (region sizes use the full tile size T, ragged tiles use part of it)
    const int fx = T[0] + 2 * H, fy = T[1] + 2 * H, fz = T[2] + 2 * H;
    const int fpl = field_plane(fx, fy);
    const int fr = fpl * fz;
    const int jx = T[0] + 2 * guard + 5, jy = T[1] + 2 * guard + 5, jz = T[2] + 2 * guard + 5;
    const int jpl = cur_plane(jx, jy);
    const int jr = jpl * jz;
    unsigned long long* Jl = lds_u64;
    float* Fl = reinterpret_cast<float*>(lds_u64 + 3 * jr);

    for (int i = threadIdx.x; i < 3 * jr; i += NT) Jl[i] = 0ull;
    // stage E, B (tile + halo, periodic wrap in storage coordinates); note
    // whether any staged value is other than +0
    unsigned int bits = 0u;
    for (int i = threadIdx.x; i < fx * fy * fz; i += NT) {
        const int lz = i / (fx * fy);
        const int rr = i - lz * fx * fy;
        const int ly = rr / fx;
        const int lx = rr - ly * fx;
        int gx = t0[0] - H + lx, gy = t0[1] - H + ly, gz = t0[2] - H + lz;
        gx = wrap_any(gx, g.n[0]);
        gy = wrap_any(gy, g.n[1]);
        gz = wrap_any(gz, g.n[2]);
        const int gi = gx + g.n[0] * (gy + g.n[1] * gz);
        const int li = lz * fpl + rr;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = f.E[c][gi], b = f.B[c][gi];
            Fl[c * fr + li] = e;
            Fl[(3 + c) * fr + li] = b;
            bits |= __float_as_uint(e) | __float_as_uint(b);
        }
    }
    // A cold tile: every staged field value is +0 (ahead of the laser).  There a
    // particle with u = +0 gathers E = B = +0, and the push, move and deposit
    // leave it exactly as it is (u stays +0, the offsets and the cell do not
    // change, nothing moves so nothing is deposited): it is skipped.
    const bool cold_tile = __syncthreads_or(bits != 0u) == 0;

    float* const El[3] = {Fl, Fl + fr, Fl + 2 * fr};
    float* const Bl[3] = {Fl + 3 * fr, Fl + 4 * fr, Fl + 5 * fr};
    const int fstride[3] = {1, fx, fpl};
    const int jstride[3] = {1, jx, jpl};
    const int pb = toff[tile];
    const int n = toff[tile + 1] - pb;
    int errs = 0;
    // software pipeline: the next particle's SoA loads are issued before the
    // current particle is processed
    int pn = pb + (int)threadIdx.x, celln = -1;
    float on[3] = {0.f, 0.f, 0.f}, un[3] = {0.f, 0.f, 0.f}, wn = 0.f;
    if ((NT < 1024 || !GATHER) && (int)threadIdx.x < n) load_particle<GATHER>(s, src, pn, celln, on, un, wn);
    for (int q = threadIdx.x; q < n; q += NT) {
        if (NT >= 1024 && GATHER) {
            pn = pb + q;
            load_particle<GATHER>(s, src, pn, celln, on, un, wn);
        }
        const int p = pn;
        const int cell = celln;
        float o[3] = {on[0], on[1], on[2]};
        float u[3] = {un[0], un[1], un[2]};
        const float wq = s.mq * wn;
        // (not in the 1024-thread launch right after a sort, whose loads go
        // through the source index: measured slower there with it)
        if ((NT < 1024 || !GATHER) && q + NT < n) {
            pn = p + NT;
            load_particle<GATHER>(s, src, pn, celln, on, un, wn);
        }
        if ((unsigned)cell >= (unsigned)g.ncell) {   // (a sort drops these)
            if (GATHER) s.cell[p] = cell;
            keep_particle<GATHER>(s, p, o, u);
            continue;
        }
        int c[3];
        decompose(g, cell, c);
        if (particle_killed(g, c)) {
            s.cell[p] = -1;
            keep_particle<GATHER>(s, p, o, u);
            continue;
        }
        int lc[3];
        bool inside = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int l = c[d] - t0[d];
            if (l >= te[d] + guard) l -= g.n[d];
            if (l < -guard) l += g.n[d];
            lc[d] = l;
            inside = inside && l >= -guard && l < te[d] + guard;
        }
        if (!inside) {   // beyond the guard: the rest pass takes it
            s.cell[p] = -2 - cell;
            keep_particle<GATHER>(s, p, o, u);
            const unsigned long long m = __ballot(1);   // the lanes in this branch
            const int lane = __lane_id(), leader = __ffsll((long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(rest_n, __popcll(m));
            base = __shfl(base, leader);
            rest_idx[base + __popcll(m & ((1ull << lane) - 1ull))] = p;
            continue;
        }
        if (cold_tile && (__float_as_uint(u[0]) | __float_as_uint(u[1]) | __float_as_uint(u[2])) == 0u) {
            if (GATHER) {   // the particle still moves to its sorted place
                s.cell[p] = cell;
                keep_particle<GATHER>(s, p, o, u);
            }
            continue;
        }
        const float o0[3] = {o[0], o[1], o[2]};
        GatherStencil st;
        gather_stencil(o, st);
        float E[3], B[3];
        {
            int ii[3][4], ih[3][4];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    ii[d][a] = (lc[d] + H - 1 + a) * fstride[d];
                    ih[d][a] = (lc[d] + H + st.hb[d] + a) * fstride[d];
                }
            gather_fields(El, Bl, ii, ih, st, E, B);
        }
        int c1[3] = {c[0], c[1], c[2]};
        errs |= push_move(g, s.qmh, E, B, u, o, c1);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            s.u[d][p] = u[d];
            s.off[d][p] = o[d];
        }
        s.cell[p] = c1[0] + g.n[0] * (c1[1] + g.n[1] * c1[2]);
        if (!moved(c, c1, o0, o)) continue;   // every contribution would be zero
        Axis5 A[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) axis5(unwrap_shift(c1[d] - c[d], g.n[d]), o0[d], o[d], A[d]);
        LdsEmit em;
        em.base = Jl + ((lc[0] + guard + 1) + (lc[1] + guard + 1) * jstride[1] + (lc[2] + guard + 1) * jstride[2]);
        em.jx = jstride[1];
        em.jpl = jstride[2];
        em.jr = jr;
        // backward crossing: the transverse extra slot moves from +4 to -1
        // slots, the own-axis one from +3 to -1
        em.dxm = A[0].base < -1 ? -5 : 0;
        em.dxp = A[0].base < -1 ? -4 : 0;
        em.dym = A[1].base < -1 ? -5 * jstride[1] : 0;
        em.dyp = A[1].base < -1 ? -4 * jstride[1] : 0;
        em.dzm = A[2].base < -1 ? -5 * jstride[2] : 0;
        em.dzp = A[2].base < -1 ? -4 * jstride[2] : 0;
        esirkepov<true>(A, wq, em);
    }
    if (errs) atomicOr(d_err, errs);
    __syncthreads();
    // flush the non-zero LDS current into the global accumulator
    const int lo = guard + 2;
    for (int i = threadIdx.x; i < 3 * jr; i += NT) {
        const unsigned long long v = Jl[i];
        if (v == 0ull) continue;   // (the padding of each plane stays zero)
        const int comp = i / jr;
        const int k = i - comp * jr;
        const int lz = k / jpl;
        const int rr = k - lz * jpl;
        const int ly = rr / jx;
        const int lx = rr - ly * jx;
        int gx = t0[0] - lo + lx, gy = t0[1] - lo + ly, gz = t0[2] - lo + lz;
        gx = wrap_any(gx, g.n[0]);
        gy = wrap_any(gy, g.n[1]);
        gz = wrap_any(gz, g.n[2]);
        atomicAdd(acc + ((size_t)comp * g.ncell + gx + g.n[0] * (gy + g.n[1] * gz)), v);
    }
}

template <int NT, int TX = 0, int TY = 0, int TZ = 0, int GD = -1, bool GATHER = false>
__global__ void __launch_bounds__(NT) k_pic_tile(Geom g, TileGeom t, int guard, FieldPtrs f, SpeciesDev s,
                                                 SpeciesDev src, const int* __restrict__ toff,
                                                 unsigned long long* __restrict__ acc, int* __restrict__ d_err,
                                                 int* __restrict__ rest_n, int* __restrict__ rest_idx) {
    extern __shared__ unsigned long long lds_u64[];
    const int tile = xcd_tile(blockIdx.x, t.ntiles, t.nt[0]);
    if (tile >= t.ntiles) return;
    tile_body<NT, TX, TY, TZ, GD, GATHER>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, lds_u64,
                                          tile);
}

// Batched form: the work list is the concatenation of every member's tiles
// (member m owns flat tiles [tile_begin[m], tile_begin[m+1])), mapped XCD by
// XCD like the single-instance launch.  TX..GD > 0 (>= 0): every member has
// that tile shape and guard (the compile-time body of the single launch).
template <int NT, int TX = 0, int TY = 0, int TZ = 0, int GD = -1>
__global__ void __launch_bounds__(NT) k_batch_tile(const InstDesc* __restrict__ tab,
                                                   const int* __restrict__ tile_begin, int n, int total) {
    extern __shared__ unsigned long long lds_u64[];
    const int ft = xcd_tile(blockIdx.x, total, kBatchChunk);
    if (ft >= total) return;
    int lo = 0, hi = n - 1;   // last member whose range starts at or before ft
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_begin[mid] <= ft) lo = mid; else hi = mid - 1;
    }
    const InstDesc& d = tab[lo];
    const Geom g = d.g;
    const TileGeom t = d.t;
    const FieldPtrs f = d.f;
    const SpeciesDev s = step_arrays(d);
    // a member that sorted this step gathers its particles from the pre-sort set
    if (d.sorting)
        tile_body<NT, TX, TY, TZ, GD, true>(g, t, d.guard, f, s, d.s, d.toff, d.acc, d.err, d.rest_n, d.rank, lds_u64,
                                            ft - tile_begin[lo]);
    else
        tile_body<NT, TX, TY, TZ, GD>(g, t, d.guard, f, s, s, d.toff, d.acc, d.err, d.rest_n, d.rank, lds_u64,
                                      ft - tile_begin[lo]);
}

// The rest pass, after the tile kernel: the particles on the species' rest
// list (marked by the tile kernel with cell -2 - c) and those appended after
// the last sort (index >= sorted, in no tile range) take the same step
// through global memory.  Item i < n_rest is list entry i, item n_rest + j
// is particle sorted + j.
__device__ __forceinline__ void rest_item(const Geom& g, const FieldPtrs& f, const SpeciesDev& s, int i, int nrest,
                                          int sorted, const int* __restrict__ rest_idx,
                                          unsigned long long* acc, int* d_err) {
    int p, c[3];
    if (i < nrest) {
        p = rest_idx[i];
        decompose(g, -2 - s.cell[p], c);   // the tile kernel already applied the window cut
    } else {
        p = sorted + (i - nrest);
        const int cell = s.cell[p];
        if ((unsigned)cell >= (unsigned)g.ncell) return;
        decompose(g, cell, c);
        if (particle_killed(g, c)) {
            s.cell[p] = -1;
            return;
        }
    }
    const int errs = push_deposit_global(g, f, s, p, c, acc);
    if (errs) atomicOr(d_err, errs);
}

constexpr int kRestThreads = 256;

__global__ void __launch_bounds__(kRestThreads) k_tile_rest(Geom g, FieldPtrs f, SpeciesDev s,
                                                            const int* __restrict__ d_sorted,
                                                            const int* __restrict__ d_count,
                                                            const int* __restrict__ rest_n,
                                                            const int* __restrict__ rest_idx,
                                                            unsigned long long* __restrict__ acc,
                                                            int* __restrict__ d_err) {
    const int nrest = *rest_n, sorted = *d_sorted;
    const int total = nrest + max(0, *d_count - sorted);
    for (int i = blockIdx.x * kRestThreads + threadIdx.x; i < total; i += gridDim.x * kRestThreads)
        rest_item(g, f, s, i, nrest, sorted, rest_idx, acc, d_err);
}

__global__ void __launch_bounds__(kRestThreads) k_batch_rest(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const Geom g = d.g;
    const FieldPtrs f = d.f;
    const SpeciesDev s = step_arrays(d);
    const int nrest = *d.rest_n, sorted = *d.sorted;
    const int total = nrest + max(0, *d.count - sorted);
    for (int i = blockIdx.x * kRestThreads + threadIdx.x; i < total; i += gridDim.x * kRestThreads)
        rest_item(g, f, s, i, nrest, sorted, d.rank, d.acc, d.err);
}

// Rest-list counters start at zero before each tile launch (a kernel, not a
// memset, so that a captured step stays valid).
__global__ void k_zero_rest(int* rest_n) { *rest_n = 0; }

__global__ void k_batch_zero_rest(const InstDesc* __restrict__ tab, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *tab[i].rest_n = 0;
}

size_t tile_lds_bytes(const TileGeom& t, int guard) {
    const int H = guard + 2;
    const size_t fr = (size_t)field_plane(t.T[0] + 2 * H, t.T[1] + 2 * H) * (t.T[2] + 2 * H);
    const size_t jr = (size_t)cur_plane(t.T[0] + 2 * guard + 5, t.T[1] + 2 * guard + 5) * (t.T[2] + 2 * guard + 5);
    return 3 * jr * 8 + 6 * fr * 4;
}

template <int NT, int TX, int TY, int TZ, int GD, bool GATHER>
static hipError_t launch_tile_k(const Geom& g, const TileGeom& t, int guard, const FieldPtrs& f,
                                const SpeciesDev& s, const SpeciesDev& src, const int* toff, unsigned long long* acc,
                                int* d_err, int* rest_n, int* rest_idx, hipStream_t st) {
    const size_t lds = tile_lds_bytes(t, guard);
    const int nb = xcd_blocks(t.ntiles, t.nt[0]);
    hipError_t e = hipFuncSetAttribute((const void*)k_pic_tile<NT, TX, TY, TZ, GD, GATHER>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_rest, dim3(1), dim3(1), 0, st, rest_n);
    hipLaunchKernelGGL((k_pic_tile<NT, TX, TY, TZ, GD, GATHER>), dim3(nb), dim3(NT), lds, st, g, t, guard, f, s, src,
                       toff, acc, d_err, rest_n, rest_idx);
    return hipGetLastError();
}

template <int NT, int TX = 0, int TY = 0, int TZ = 0, int GD = -1>
static hipError_t launch_tile_nt(const Geom& g, const TileGeom& t, int guard, const FieldPtrs& f,
                                 const SpeciesDev& s, const SpeciesDev* src, const int* toff, unsigned long long* acc,
                                 int* d_err, int* rest_n, int* rest_idx, hipStream_t st) {
    if (src)
        return launch_tile_k<NT, TX, TY, TZ, GD, true>(g, t, guard, f, s, *src, toff, acc, d_err, rest_n, rest_idx, st);
    return launch_tile_k<NT, TX, TY, TZ, GD, false>(g, t, guard, f, s, s, toff, acc, d_err, rest_n, rest_idx, st);
}

// Tile shapes with a compile-time specialisation (the library default and
// the autotuner's usual picks); every other shape runs the general body.
template <int NT>
static hipError_t launch_tile_shape(const Geom& g, const TileGeom& t, int guard, const FieldPtrs& f,
                                    const SpeciesDev& s, const SpeciesDev* src, const int* toff,
                                    unsigned long long* acc, int* d_err, int* rest_n, int* rest_idx, hipStream_t st) {
    if (t.T[0] == 8 && t.T[1] == 8 && t.T[2] == 8) {
        if (guard == 1)
            return launch_tile_nt<NT, 8, 8, 8, 1>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, st);
        if (guard == 0)
            return launch_tile_nt<NT, 8, 8, 8, 0>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, st);
    }
    if (t.T[0] == 8 && t.T[1] == 8 && t.T[2] == 4 && guard == 1)
        return launch_tile_nt<NT, 8, 8, 4, 1>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, st);
    return launch_tile_nt<NT>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, st);
}

hipError_t launch_pic_tile(const Geom& g, const TileGeom& t, int guard, int threads, const FieldPtrs& f,
                           const SpeciesDev& s, const SpeciesDev* src, const int* toff, unsigned long long* acc,
                           int* d_err, int* rest_n, int* rest_idx, hipStream_t st) {
    switch (threads) {
        case 256: return launch_tile_shape<256>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, st);
        case 1024: return launch_tile_shape<1024>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, st);
        default: return launch_tile_shape<512>(g, t, guard, f, s, src, toff, acc, d_err, rest_n, rest_idx, st);
    }
}

template <int NT, int TX = 0, int TY = 0, int TZ = 0, int GD = -1>
static hipError_t launch_batch_tile_k(const InstDesc* d, const int* tile_begin, int n, int total, size_t lds,
                                      hipStream_t st) {
    const int nb = xcd_blocks(total, kBatchChunk);
    hipError_t e = hipFuncSetAttribute((const void*)k_batch_tile<NT, TX, TY, TZ, GD>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_zero_rest, dim3((n + 63) / 64), dim3(64), 0, st, d, n);
    hipLaunchKernelGGL((k_batch_tile<NT, TX, TY, TZ, GD>), dim3(nb), dim3(NT), lds, st, d, tile_begin, n, total);
    return hipGetLastError();
}

template <int NT>
static hipError_t launch_batch_tile_nt(const InstDesc* d, const int* tile_begin, int n, int total, size_t lds,
                                       bool all_888g1, hipStream_t st) {
    if (all_888g1) return launch_batch_tile_k<NT, 8, 8, 8, 1>(d, tile_begin, n, total, lds, st);
    return launch_batch_tile_k<NT>(d, tile_begin, n, total, lds, st);
}

hipError_t launch_batch_tile(const InstDesc* d, const int* tile_begin, int n, int total_tiles, int threads,
                             size_t lds_bytes, bool all_888g1, hipStream_t st) {
    if (n <= 0 || total_tiles <= 0) return hipSuccess;
    switch (threads) {
        case 256: return launch_batch_tile_nt<256>(d, tile_begin, n, total_tiles, lds_bytes, all_888g1, st);
        case 1024: return launch_batch_tile_nt<1024>(d, tile_begin, n, total_tiles, lds_bytes, all_888g1, st);
        default: return launch_batch_tile_nt<512>(d, tile_begin, n, total_tiles, lds_bytes, all_888g1, st);
    }
}

// Rest pass grids: a fixed number of blocks walking the items (list entries
// plus appended particles, a small share of the species in a step).
hipError_t launch_batch_rest(const InstDesc* d, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_rest, dim3(std::max(1, 1024 / n), n), dim3(kRestThreads), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_tile_rest(const Geom& g, const FieldPtrs& f, const SpeciesDev& s, const int* d_sorted,
                            const int* d_count, const int* rest_n, const int* rest_idx, unsigned long long* acc,
                            int* d_err, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_rest, dim3(1024), dim3(kRestThreads), 0, st, g, f, s, d_sorted, d_count, rest_n,
                       rest_idx, acc, d_err);
    return hipGetLastError();
}

}  // namespace pic
