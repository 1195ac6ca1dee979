// Counting sort of particles into tiles of Tx x Ty x Tz cells.
//
// Key of a particle = tile-major cell index: tile * Tcells + local cell (in
// 8x2x4-cell bricks where the tile shape allows, see local_key).  A
// histogram over keys (int atomics; the returned value is the particle's rank
// within its cell), an exclusive scan of the histogram, a scatter of each
// particle's index to its destination and a gather of the particle data by
// destination place every tile's particles contiguously.  Removed particles
// (cell < 0, or outside a moving window) are dropped.  Inside the production
// step the gather is left to the tile kernel that runs next (it reads each
// particle through the source index and writes all its arrays), which saves
// the copy pass's read and write of every particle.
//
// Order inside a tile.  Depth 0 (level order): level r holds the (r + 1)-th
// particle of every cell of the tile that has one, cells in key order, and
// the levels follow each other; the 64 lanes of a wavefront that reads the
// tile in order then sit in 64 distinct cells, consecutive cells of one
// level, whatever the density (where cells hold unequal counts, a transpose
// puts several lanes of one atomic pass in one cell, and LDS atomics to one
// address serialise).  Depth D >= 1: the cell-sorted sequence is stored
// block-transposed: each full block of 64*D particles is written as a D x 64
// transpose, so the lanes see particles D apart in cell order (different
// cells where a cell holds D particles); D = 1 is plain cell order.  Either
// way the loads stay coalesced, and particles that kept their cell since the
// last sort mostly keep their place, so the gather is close to a streaming
// copy.
#include "pic_internal.h"
#include "pic_particle_ops.h"

namespace pic {

// Cell order inside a tile: for tiles of 8 x 2m x 4k cells, 64-cell bricks
// of 8x2x4 cells (x fastest, then z, then y inside a brick; bricks y-major),
// so that a wavefront reading 64 consecutive cells of a level (or one
// transposed block) of such a brick has its lanes in 8 x-cells of
// successive z-planes (the tile kernel pads its LDS planes to match); plain
// x-fastest order for every other shape.
__device__ __forceinline__ int local_key(const TileGeom& t, int lx, int ly, int lz) {
    if (t.T[0] == 8 && (t.T[1] & 1) == 0 && (t.T[2] & 3) == 0)
        return lx + 8 * (lz & 3) + 32 * (ly & 1) + 64 * ((ly >> 1) + (t.T[1] >> 1) * (lz >> 2));
    return lx + t.T[0] * (ly + t.T[1] * lz);
}

__device__ __forceinline__ int tile_key(const TileGeom& t, const SortDiv& sd, const int c[3]) {
    const int tx = fdiv(c[0], sd.T[0]), ty = fdiv(c[1], sd.T[1]), tz = fdiv(c[2], sd.T[2]);
    const int lx = c[0] - tx * t.T[0], ly = c[1] - ty * t.T[1], lz = c[2] - tz * t.T[2];
    const int tile = tx + t.nt[0] * (ty + t.nt[1] * tz);
    return tile * t.tcells + local_key(t, lx, ly, lz);
}

// cell -> (x, y, z) for 0 <= cl < ncell, by the precomputed divisors
__device__ __forceinline__ void cell_coords(const Geom& g, const SortDiv& sd, int cl, int c[3]) {
    const int cz = fdiv(cl, sd.nxy);
    const int r = cl - cz * g.nxy;
    const int cy = fdiv(r, sd.nx);
    c[0] = r - cy * g.n[0];
    c[1] = cy;
    c[2] = cz;
}

__device__ __forceinline__ int sort_key(const Geom& g, const TileGeom& t, const SortDiv& sd, int cl) {
    if ((unsigned)cl >= (unsigned)g.ncell) return -1;
    int c[3];
    cell_coords(g, sd, cl, c);
    if (particle_killed(g, c)) return -1;
    return tile_key(t, sd, c);
}

// Histogram and rank of the kCountRows particles p0 + S r (r = 0..7), S the
// row stride: after a transposing sort (S = 64) these are the rows of one
// lane of a transposed block, after a level-order sort (S = cells per tile)
// the same cell on successive levels where the levels are full; mostly the
// particles of one cell, so one atomic per distinct key serves them all and
// the ranks follow the row order (particles that kept their cell then mostly
// keep their place, which keeps the scatter's stores coalesced).  Any
// grouping is correct: a rank is a place among the particles of one key.
constexpr int kCountRows = 8;

// foreign: the ranks are places among a key's incoming particles of a
// re-sort (after the key's local ones, see k_sort_count_tiles): stored as
// -2 - rank.
__device__ __forceinline__ void count_column(const Geom& g, const TileGeom& t, const SortDiv& sd,
                                             const int* __restrict__ cell, int p0, int stride, bool foreign,
                                             int n, int* __restrict__ hist, int* __restrict__ rank) {
    int key[kCountRows];
#pragma unroll
    for (int r = 0; r < kCountRows; ++r) {
        const int p = p0 + stride * r;
        key[r] = p < n ? sort_key(g, t, sd, cell[p]) : -2;
    }
    int rk[kCountRows];
#pragma unroll
    for (int r = 0; r < kCountRows; ++r) rk[r] = -1;
#pragma unroll
    for (int r = 0; r < kCountRows; ++r) {
        if (key[r] < 0 || rk[r] >= 0) continue;   // removed, or ranked with an earlier row
        int cnt = 0;
#pragma unroll
        for (int q = r; q < kCountRows; ++q) cnt += key[q] == key[r];
        int base = atomicAdd(hist + key[r], cnt);
#pragma unroll
        for (int q = r; q < kCountRows; ++q)
            if (key[q] == key[r]) rk[q] = base++;
    }
#pragma unroll
    for (int r = 0; r < kCountRows; ++r) {
        const int p = p0 + stride * r;
        if (p < n) rank[p] = foreign && rk[r] >= 0 ? -2 - rk[r] : rk[r];
    }
}

// Row stride of the count for a sort of the given depth, and the column of
// thread i: p0 = (i / S) * 8 S + i % S.
__host__ __device__ __forceinline__ int count_stride(const TileGeom& t, int depth) {
    return depth == 0 ? t.tcells : 64;
}
__device__ __forceinline__ int column_of(int i, int stride) {
    const int b = i / stride;
    return b * (stride * kCountRows) + (i - b * stride);
}
// threads that cover n particles in whole blocks of columns
inline int count_threads(int n, int stride) {
    const int blk = stride * kCountRows;
    return (n + blk - 1) / blk * stride;
}

// Columns over particles [*d_begin, *d_count) (d_begin null: from 0).
__global__ void __launch_bounds__(256) k_sort_count(Geom g, TileGeom t, SortDiv sd, const int* __restrict__ cell,
                                                    const int* __restrict__ d_begin, const int* __restrict__ d_count,
                                                    int stride, int foreign, int* __restrict__ hist,
                                                    int* __restrict__ rank) {
    const int p0 = (d_begin ? *d_begin : 0) + column_of(blockIdx.x * blockDim.x + threadIdx.x, stride);
    const int n = *d_count;
    if (p0 >= n) return;
    count_column(g, t, sd, cell, p0, stride, foreign != 0, n, hist, rank);
}

// Count pass of a re-sort over the particles that the last sort put in tile
// ranges: workgroup b takes tile b's old range [toff[b], toff[b + 1]).  Most
// of them are still in that tile (they move less than a cell per step): they
// are ranked in an LDS histogram of the tile's keys (local ranks 0 .. lc - 1,
// lc[key] stored for every key of the tile), with no global atomic.  A
// particle that left its tile (and every particle appended since the sort)
// takes a place among the key's incoming particles from the global
// histogram, stored as -2 - place, and goes after the key's local ones
// (rank lc[key] + place, resolved by the scatter); removed ones get -1.  The
// histogram then adds lc: every key's count is complete and every rank unique.
constexpr int kTileCountThreads = 512;

__device__ __forceinline__ void count_tile(const Geom& g, const TileGeom& t, const SortDiv& sd,
                                           const int* __restrict__ cell, const int* __restrict__ toff,
                                           int* __restrict__ hist, int* __restrict__ lc, int* __restrict__ rank,
                                           int tile, int* lh) {
    const int k0 = tile * t.tcells;
    for (int i = threadIdx.x; i < t.tcells; i += kTileCountThreads) lh[i] = 0;
    __syncthreads();
    const int b = toff[tile], e = toff[tile + 1];
    // four particles per thread at a time, their cells loaded together
    for (int p0 = b + (int)threadIdx.x; p0 < e; p0 += 4 * kTileCountThreads) {
        int cl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = p0 + u * kTileCountThreads;
            cl[u] = p < e ? cell[p] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = p0 + u * kTileCountThreads;
            if (p >= e) continue;
            const int key = sort_key(g, t, sd, cl[u]);
            int r = -1;
            if ((unsigned)(key - k0) < (unsigned)t.tcells) r = atomicAdd(&lh[key - k0], 1);
            else if (key >= 0) r = -2 - atomicAdd(&hist[key], 1);
            rank[p] = r;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < t.tcells; i += kTileCountThreads) lc[k0 + i] = lh[i];
}

__global__ void __launch_bounds__(kTileCountThreads) k_sort_count_tiles(Geom g, TileGeom t, SortDiv sd,
                                                                        const int* __restrict__ cell,
                                                                        const int* __restrict__ toff,
                                                                        int* __restrict__ hist, int* __restrict__ lc,
                                                                        int* __restrict__ rank) {
    extern __shared__ int lh[];   // t.tcells counters
    count_tile(g, t, sd, cell, toff, hist, lc, rank, blockIdx.x, lh);
}

__global__ void __launch_bounds__(256) k_add_counts(int* __restrict__ hist, const int* __restrict__ lc, int nkeys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nkeys) hist[i] += lc[i];
}

// Level order of one tile (depth 0).  The scatter has stored the tile's
// source indices in plain cell order in `src` (off[key] is the first
// cell-order place of a key, off[key + 1] - off[key] its count); this writes
// them to `out` in level order: the (r + 1)-th particle of key k goes to the
// tile's start, plus the sizes of levels 0..r-1, plus the number of keys
// before k holding more than r particles.  Consecutive keys of a level write
// consecutive places (coalesced stores); the tile's cell-order slice is read
// through LDS when it fits.  One workgroup per tile; thread i owns keys
// i per .. i per + per - 1; one barrier per level (the wave totals alternate
// between two LDS rows).
constexpr int kLevelThreads = 512;
constexpr int kLevelMaxPer = 8;      // tiles of up to 4096 cells
constexpr int kLevelStage = 8192;    // particles of a tile staged in LDS
constexpr int kPlaceUnroll = 4;

// The particles that stayed in a tile since the last sort (a re-sort, see
// k_sort_count_tiles): workgroup `tile` also reads its old range [ob, oe)
// and puts each particle of rank r >= 0 (it stayed, so its key is in this
// tile) straight at its cell-order place -- in LDS, or in `src` for a tile too
// large to stage -- so that only the particles that changed tile go through
// the scatter (see k_sort_scatter_moved); lc[key] of a key's places are
// local, the rest are read from `src`.
struct LocalPlace {
    Geom g;
    TileGeom t;
    SortDiv sd;
    const int* cell;
    const int* rank;
    const int* toff;   // the last sort's tile ranges
    const int* lc;
};

__device__ __forceinline__ void sort_levels_tile(const int* __restrict__ off, int tcells, int* __restrict__ src,
                                                 int* __restrict__ out, int tile,
                                                 const LocalPlace* __restrict__ lp = nullptr) {
    __shared__ int wsum[2][kLevelThreads / 64];
    __shared__ int stage[kLevelStage];
    const int base = tile * tcells;
    const int per = (tcells + kLevelThreads - 1) / kLevelThreads;
    const int k0 = (int)threadIdx.x * per;
    const int tb = off[base];
    const int n = off[base + tcells] - tb;
    const bool staged = n <= kLevelStage;
    int start[kLevelMaxPer], cnt[kLevelMaxPer];
    int cmax = 0;
#pragma unroll
    for (int j = 0; j < kLevelMaxPer; ++j) {
        const int k = k0 + j;
        start[j] = 0;
        cnt[j] = 0;
        if (j < per && k < tcells) {
            start[j] = off[base + k] - tb;
            cnt[j] = off[base + k + 1] - tb - start[j];
            cmax = max(cmax, cnt[j]);
        }
    }
    if (lp) {
        const int ob = lp->toff[tile], oe = lp->toff[tile + 1];
        // kPlaceUnroll particles per thread at a time, each stage's loads
        // issued for all of them before any is used (the chain rank, cell ->
        // key -> off[key] is otherwise one round trip after another)
        constexpr int U = kPlaceUnroll;
        for (int p0 = ob + (int)threadIdx.x; p0 < oe; p0 += U * kLevelThreads) {
            int r[U], cl[U], o[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = p0 + u * kLevelThreads;
                r[u] = p < oe ? lp->rank[p] : -1;
                cl[u] = p < oe ? lp->cell[p] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                o[u] = 0;
                if (r[u] >= 0) {   // (r < 0: removed, or moved to another tile)
                    int c[3];
                    cell_coords(lp->g, lp->sd, cl[u], c);
                    o[u] = off[tile_key(lp->t, lp->sd, c)];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (r[u] < 0) continue;
                const int slot = o[u] - tb + r[u];
                if (staged) stage[slot] = p0 + u * kLevelThreads;
                else src[tb + slot] = p0 + u * kLevelThreads;   // (read back by this workgroup after the barrier)
            }
        }
        if (staged)
#pragma unroll
            for (int j = 0; j < kLevelMaxPer; ++j)
                if (j < per && k0 + j < tcells)
                    for (int q = lp->lc[base + k0 + j]; q < cnt[j]; ++q) stage[start[j] + q] = src[tb + start[j] + q];
    } else if (staged) {
        for (int i = threadIdx.x; i < n; i += kLevelThreads) stage[i] = src[tb + i];
    }
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    int lbase = tb;
    bool more = __syncthreads_or(cmax > 0) != 0;   // (also: the staged slice is complete)
    for (int r = 0; more; ++r) {
        int mine = 0;
#pragma unroll
        for (int j = 0; j < kLevelMaxPer; ++j) mine += cnt[j] > r;
        int incl;   // inclusive prefix of `mine` over the wavefront
        if (per == 1) {
            incl = __popcll(__ballot(mine != 0) << (63 - lane));
        } else {
            incl = mine;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
        }
        if (lane == 63) wsum[r & 1][wv] = incl;
        more = __syncthreads_or(cmax > r + 1) != 0;
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kLevelThreads / 64; ++w) {
            const int v = wsum[r & 1][w];
            total += v;
            before += w < wv ? v : 0;
        }
        int pos = lbase + before + incl - mine;
#pragma unroll
        for (int j = 0; j < kLevelMaxPer; ++j)
            if (cnt[j] > r) out[pos++] = staged ? stage[start[j] + r] : src[tb + start[j] + r];
        lbase += total;
    }
}

__global__ void __launch_bounds__(kLevelThreads) k_sort_levels(const int* __restrict__ off, int tcells,
                                                               int* __restrict__ src, int* __restrict__ out) {
    sort_levels_tile(off, tcells, src, out, blockIdx.x);
}

__global__ void __launch_bounds__(kLevelThreads) k_sort_levels_local(const int* __restrict__ off, int tcells,
                                                                     int* __restrict__ src, int* __restrict__ out,
                                                                     LocalPlace lp) {
    sort_levels_tile(off, tcells, src, out, blockIdx.x, &lp);
}

// Exclusive scan, phase 1: per-block totals of 1024-element blocks.
__device__ __forceinline__ void scan_reduce_block(const int* __restrict__ in, int n, int* __restrict__ sums, int bx) {
    __shared__ int ws[16];
    const int i = bx * 1024 + threadIdx.x;
    int v = i < n ? in[i] : 0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int k = 0; k < 16; ++k) s += ws[k];
        sums[bx] = s;
    }
}

__global__ void __launch_bounds__(1024) k_scan_reduce(const int* __restrict__ in, int n, int* __restrict__ sums) {
    scan_reduce_block(in, n, sums, blockIdx.x);
}

// Block-wide inclusive scan of one value per thread (1024 threads).
__device__ __forceinline__ int block_scan_incl(int v, int* ws) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    if (lane == 63) ws[wv] = v;
    __syncthreads();
    if (threadIdx.x < 16) {
        int s = ws[threadIdx.x];
        for (int o = 1; o < 16; o <<= 1) {
            const int y = __shfl_up(s, o, 16);
            if ((threadIdx.x & 15) >= o) s += y;
        }
        ws[16 + threadIdx.x] = s;
    }
    __syncthreads();
    const int add = wv > 0 ? ws[16 + wv - 1] : 0;
    __syncthreads();
    return v + add;
}

// Phase 2: exclusive scan of the block totals by one workgroup; total -> sums[nb].
__device__ __forceinline__ void scan_sums_block(int* __restrict__ sums, int nb) {
    __shared__ int ws[32];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? sums[i] : 0;
        const int inc = block_scan_incl(v, ws);
        const int c0 = carry;
        if (i < nb) sums[i] = c0 + inc - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry = c0 + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(1024) k_scan_sums(int* __restrict__ sums, int nb) { scan_sums_block(sums, nb); }

// Phase 3: exclusive scan inside each block plus the block offset; out may alias in.
__device__ __forceinline__ void scan_apply_block(const int* in, int n, const int* __restrict__ sums, int* out, int bx) {
    __shared__ int ws[32];
    const int i = bx * 1024 + threadIdx.x;
    const int v = i < n ? in[i] : 0;
    const int inc = block_scan_incl(v, ws);
    if (i < n) out[i] = sums[bx] + inc - v;
}

__global__ void __launch_bounds__(1024) k_scan_apply(const int* in, int n, const int* __restrict__ sums, int* out) {
    scan_apply_block(in, n, sums, out, blockIdx.x);
}

// Source index of particle p to its place: out[off[key] + rank] in cell
// order (an incoming particle of a re-sort, rank -2 - place, after the key's
// lc[key] local ones), then the block transpose of depth > 1.  Depth 0 (level
// order) stores cell order here; the level pass reorders it.
__device__ __forceinline__ void scatter_one(const Geom& g, const TileGeom& t, const SortDiv& sd,
                                            const int* __restrict__ src_cell, int* __restrict__ out, int p,
                                            const int* __restrict__ rank, const int* __restrict__ off,
                                            const int* __restrict__ lc, int depth) {
    int r = rank[p];
    if (r == -1) return;
    const int cl = src_cell[p];   // a ranked particle has a live cell
    int c[3];
    cell_coords(g, sd, cl, c);
    const int key = tile_key(t, sd, c);
    if (r < -1) r = lc[key] + (-2 - r);
    int dest = off[key] + r;
    if (depth > 1) {
        const int tile = fdiv(key, sd.tcells);
        const int tb = off[tile * t.tcells];
        const int j = dest - tb;
        if ((depth & (depth - 1)) == 0) {   // the usual depths: shifts
            const int sh = 6 + __ffs(depth) - 1;   // log2 of the block of 64 depth particles
            const int nfull = ((off[(tile + 1) * t.tcells] - tb) >> sh) << sh;
            if (j < nfull) {
                const int b0 = (j >> sh) << sh, k = j - b0;
                dest = tb + b0 + (k & (depth - 1)) * 64 + (k >> (sh - 6));
            }
        } else {
            const int blk = 64 * depth;
            const int nfull = (off[(tile + 1) * t.tcells] - tb) / blk * blk;
            if (j < nfull) {
                const int b0 = j - j % blk, k = j - b0;
                dest = tb + b0 + (k % depth) * 64 + k / depth;
            }
        }
    }
    out[dest] = p;   // the source index; the gather replaces it with the particle
}

// Re-sort in level order: only the particles that changed tile since the
// last sort, and those appended since (rank -2 - place), go to their
// cell-order place here; the level pass places the others.
__global__ void __launch_bounds__(256) k_sort_scatter_moved(Geom g, TileGeom t, SortDiv sd,
                                                            const int* __restrict__ src_cell, int* __restrict__ out,
                                                            const int* __restrict__ d_count,
                                                            const int* __restrict__ rank, const int* __restrict__ off,
                                                            const int* __restrict__ lc) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *d_count || rank[p] > -2) return;
    scatter_one(g, t, sd, src_cell, out, p, rank, off, lc, 0);
}

// Second pass of the permutation, over destinations: dst.cell[i] holds the
// source index (written by scatter_one), every array is copied from there.
// The stores are coalesced, and so are most loads (particles that kept their
// cell keep their place), where scattering all nine arrays from the source
// side would scatter every store.
__device__ __forceinline__ void gather_one(const SpeciesDev& src, const SpeciesDev& dst, int i) {
    const int p = dst.cell[i];
    dst.cell[i] = src.cell[p];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dst.off[d][i] = src.off[d][p];
        dst.u[d][i] = src.u[d][p];
    }
    dst.w[i] = src.w[p];
    dst.id[i] = src.id[p];
}

__global__ void __launch_bounds__(256) k_sort_scatter(Geom g, TileGeom t, SortDiv sd,
                                                      const int* __restrict__ src_cell, int* __restrict__ out,
                                                      const int* __restrict__ d_count, const int* __restrict__ rank,
                                                      const int* __restrict__ off, const int* __restrict__ lc,
                                                      int depth) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *d_count) return;
    scatter_one(g, t, sd, src_cell, out, p, rank, off, lc, depth);
}

__global__ void __launch_bounds__(256) k_sort_gather(SpeciesDev src, SpeciesDev dst, const int* __restrict__ off,
                                                     int nkeys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= off[nkeys]) return;
    gather_one(src, dst, i);
}

// New live count = total of the histogram.
__global__ void k_sort_finish(const int* __restrict__ off, int nkeys, int* __restrict__ d_count,
                              int* __restrict__ d_sorted) {
    d_count[0] = off[nkeys];
    d_sorted[0] = off[nkeys];
}

// Tile ranges of the species: toff[t] = first particle of tile t (t = 0..ntiles).
__global__ void __launch_bounds__(256) k_tile_offsets(const int* __restrict__ off, int tcells, int ntiles,
                                                      int* __restrict__ toff) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= ntiles) toff[t] = off[t * tcells];
}

// Batched sort: grid y = member; members that do not sort this step return at once.
__global__ void __launch_bounds__(256) k_batch_zero_hist(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (!d.sorting || i > d.nkeys) return;
    d.hist[i] = 0;
}

// Columns of the members that sort: all particles, or for a re-sort those
// appended since the last one (after the member's tile-by-tile count).
__global__ void __launch_bounds__(256) k_batch_sort_count(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    if (!d.sorting) return;
    const TileGeom t = d.t;
    const int stride = count_stride(t, d.depth);
    const int p0 = (d.resort ? *d.sorted : 0) + column_of(blockIdx.x * blockDim.x + threadIdx.x, stride);
    const int n = *d.count;
    if (p0 >= n) return;
    const Geom g = d.g;
    count_column(g, t, d.sdiv, d.s.cell, p0, stride, d.resort != 0, n, d.hist, d.rank);
}

// Tile-by-tile count of the members that re-sort: grid x = tile, y = member.
__global__ void __launch_bounds__(kTileCountThreads) k_batch_sort_count_tiles(const InstDesc* __restrict__ tab) {
    extern __shared__ int lh[];
    const InstDesc& d = tab[blockIdx.y];
    if (!d.sorting || !d.resort || (int)blockIdx.x >= d.t.ntiles) return;   // (uniform per workgroup)
    const Geom g = d.g;
    const TileGeom t = d.t;
    count_tile(g, t, d.sdiv, d.s.cell, d.toff, d.hist, d.lc, d.rank, blockIdx.x, lh);
}

__global__ void __launch_bounds__(256) k_batch_add_counts(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (!d.sorting || !d.resort || i >= d.nkeys) return;
    d.hist[i] += d.lc[i];
}

// Level order of the sorting members with depth 0 (after their scatter):
// grid x = tile, y = member.  A member that re-sorts places the particles
// that stayed in their tile here, from its last tile ranges (its scatter
// moved only the others), as the single simulation's re-sort does.
__global__ void __launch_bounds__(kLevelThreads) k_batch_sort_levels(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    if (!d.sorting || d.depth != 0 || (int)blockIdx.x >= d.t.ntiles) return;
    // (the workgroup returns as a whole: the condition is uniform)
    if (d.resort) {
        const LocalPlace lp{d.g, d.t, d.sdiv, d.s.cell, d.rank, d.toff, d.lc};
        sort_levels_tile(d.hist, d.t.tcells, d.level, d.alt.cell, blockIdx.x, &lp);
    } else {
        sort_levels_tile(d.hist, d.t.tcells, d.level, d.alt.cell, blockIdx.x);
    }
}

__global__ void __launch_bounds__(1024) k_batch_scan_reduce(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int n = d.nkeys + 1;
    if (!d.sorting || (int)blockIdx.x * 1024 >= n) return;
    scan_reduce_block(d.hist, n, d.sums, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_batch_scan_sums(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    if (!d.sorting) return;
    scan_sums_block(d.sums, (d.nkeys + 1 + 1023) / 1024);
}

__global__ void __launch_bounds__(1024) k_batch_scan_apply(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int n = d.nkeys + 1;
    if (!d.sorting || (int)blockIdx.x * 1024 >= n) return;
    scan_apply_block(d.hist, n, d.sums, d.hist, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_batch_sort_scatter(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (!d.sorting || p >= *d.count) return;
    // a level-order re-sort: only the particles that changed tile or were
    // appended (rank < -1); the level pass places the others
    if (d.resort && d.depth == 0 && d.rank[p] > -2) return;
    const Geom g = d.g;
    const TileGeom t = d.t;
    const SpeciesDev src = d.s, dst = d.alt;
    scatter_one(g, t, d.sdiv, src.cell, d.depth == 0 ? d.level : dst.cell, p, d.rank, d.hist, d.lc, d.depth);
}

__global__ void __launch_bounds__(256) k_batch_sort_finish(const InstDesc* __restrict__ tab) {
    const InstDesc& d = tab[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!d.sorting || t > d.t.ntiles) return;
    d.toff[t] = d.hist[t * d.t.tcells];
    if (t == 0) {
        d.count[0] = d.hist[d.nkeys];
        d.sorted[0] = d.hist[d.nkeys];
    }
}

hipError_t launch_batch_sort(const InstDesc* d, int n, int max_particles, int max_keys1, int max_tiles1,
                             int max_tcells, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int np = max_particles > 0 ? max_particles : 1;
    const int nb = (max_keys1 + 1023) / 1024;
    hipLaunchKernelGGL(k_batch_zero_hist, dim3((max_keys1 + 255) / 256, n), dim3(256), 0, st, d);
    // enough columns for every member's stride S (64, or its cells per tile):
    // whole blocks of 8 S rows need at most n / 8 + S threads
    const int ncol = (np + kCountRows - 1) / kCountRows + std::max(max_tcells, 64);
    hipLaunchKernelGGL(k_batch_sort_count_tiles, dim3(max_tiles1 - 1, n), dim3(kTileCountThreads),
                       max_tcells * sizeof(int), st, d);
    hipLaunchKernelGGL(k_batch_sort_count, dim3((ncol + 255) / 256, n), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_batch_add_counts, dim3((max_keys1 + 255) / 256, n), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_batch_scan_reduce, dim3(nb, n), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(k_batch_scan_sums, dim3(1, n), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(k_batch_scan_apply, dim3(nb, n), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(k_batch_sort_scatter, dim3((np + 255) / 256, n), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_batch_sort_levels, dim3(max_tiles1 - 1, n), dim3(kLevelThreads), 0, st, d);
    // (no copy pass: each sorting member's tile step gathers its particles)
    hipLaunchKernelGGL(k_batch_sort_finish, dim3((max_tiles1 + 255) / 256, n), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_sort(const Geom& g, const TileGeom& t, const SpeciesDev& src, const SpeciesDev& dst,
                       int* d_count, int* d_sorted, int max_count, int* hist, int* rank, int* sums, int* level,
                       int* lc, int depth, int* toff, bool copy, bool resort, hipStream_t st) {
    const int nkeys = t.ntiles * t.tcells;
    if (depth == 0 && (level == nullptr || t.tcells > kLevelThreads * kLevelMaxPer)) return hipErrorInvalidValue;
    if (resort && lc == nullptr) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(hist, 0, ((size_t)nkeys + 1) * sizeof(int), st);
    if (e != hipSuccess) return e;
    const int np = max_count > 0 ? max_count : 1;
    const int stride = count_stride(t, depth);
    const int ncol = count_threads(np, stride);
    const SortDiv sd = make_sortdiv(g, t);
    if (resort) {   // [0, *d_sorted) sit in the tile ranges toff of the last sort; appended ones after them
        hipLaunchKernelGGL(k_sort_count_tiles, dim3(t.ntiles), dim3(kTileCountThreads), t.tcells * sizeof(int), st,
                           g, t, sd, src.cell, toff, hist, lc, rank);
        hipLaunchKernelGGL(k_sort_count, dim3((ncol + 255) / 256), dim3(256), 0, st, g, t, sd, src.cell, d_sorted,
                           d_count, stride, 1, hist, rank);
        hipLaunchKernelGGL(k_add_counts, dim3((nkeys + 255) / 256), dim3(256), 0, st, hist, lc, nkeys);
    } else {
        hipLaunchKernelGGL(k_sort_count, dim3((ncol + 255) / 256), dim3(256), 0, st, g, t, sd, src.cell, nullptr,
                           d_count, stride, 0, hist, rank);
    }
    const int n = nkeys + 1;
    const int nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(1024), 0, st, hist, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, st, hist, n, sums, hist);
    if (depth == 0 && resort) {
        // toff still holds the last sort's tile ranges (rewritten at the end)
        hipLaunchKernelGGL(k_sort_scatter_moved, dim3((np + 255) / 256), dim3(256), 0, st, g, t, sd, src.cell, level,
                           d_count, rank, hist, lc);
        LocalPlace lp{g, t, sd, src.cell, rank, toff, lc};
        hipLaunchKernelGGL(k_sort_levels_local, dim3(t.ntiles), dim3(kLevelThreads), 0, st, hist, t.tcells, level,
                           dst.cell, lp);
    } else {
        hipLaunchKernelGGL(k_sort_scatter, dim3((np + 255) / 256), dim3(256), 0, st, g, t, sd, src.cell,
                           depth == 0 ? level : dst.cell, d_count, rank, hist, lc, depth);
        if (depth == 0)
            hipLaunchKernelGGL(k_sort_levels, dim3(t.ntiles), dim3(kLevelThreads), 0, st, hist, t.tcells, level,
                               dst.cell);
    }
    if (copy) hipLaunchKernelGGL(k_sort_gather, dim3((np + 255) / 256), dim3(256), 0, st, src, dst, hist, nkeys);
    hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(1), 0, st, hist, nkeys, d_count, d_sorted);
    hipLaunchKernelGGL(k_tile_offsets, dim3((t.ntiles + 1 + 255) / 256), dim3(256), 0, st, hist, t.tcells, t.ntiles,
                       toff);
    return hipGetLastError();
}

}  // namespace pic
