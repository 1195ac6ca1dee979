// Host side of the C ABI declared in include/pic.h: descriptor validation,
// workspace layout, context state and the launch sequences of each call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_internal.h"

using namespace pic;

namespace {

constexpr int kMaxSpecies = 8;
constexpr size_t kAlign = 256;
constexpr int kKillMargin = 3;   // window cells behind which particles are removed
constexpr size_t kMaxLds = 160 * 1024;
constexpr int kDiagBins = 2048;                                   // most spectrum bins
constexpr size_t kDiagWords = 64;                                 // reduction words of the diagnostics
constexpr size_t kDiagBytesFixed = (2 * kDiagBins + kDiagWords) * 8;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Resolved tiling parameters of a descriptor (defaults applied).
struct Tiling {
    TileGeom t;
    int guard, threads, interleave, sort_interval;
};

Tiling tiling_of(const pic_grid_desc* d) {
    Tiling r;
    for (int a = 0; a < 3; ++a) {
        int T = d->tile[a] > 0 ? d->tile[a] : 8;
        if (T > d->n[a]) T = d->n[a];
        r.t.T[a] = T;
        r.t.nt[a] = (d->n[a] + T - 1) / T;
    }
    r.t.ntiles = r.t.nt[0] * r.t.nt[1] * r.t.nt[2];
    r.t.tcells = r.t.T[0] * r.t.T[1] * r.t.T[2];
    r.guard = d->guard < 0 ? 1 : d->guard;
    r.threads = d->threads > 0 ? d->threads : 512;
    r.interleave = d->interleave > 0 ? d->interleave : 0;   // 0: level order
    r.sort_interval = d->sort_interval > 0 ? d->sort_interval : 2;
    return r;
}

// Device workspace carve-up.  Per-particle arrays have max_particles entries;
// species take consecutive sub-ranges of them.
struct Layout {
    size_t acc, jtmp, rho, small, prev_cell, prev_off, alt_cell, alt_off, alt_u, alt_w, alt_id, sort_rank, hist, sort_lc,
        sums, toff, toff_stride, dn_w, dn_h1, dn_h2, diag, total;
};

// small block: err flags, per-species counts, reduction results
struct Small {
    int err;
    int pad0;
    int count[kMaxSpecies];    // live + removed-but-not-yet-dropped particles
    int sorted[kMaxSpecies];   // particles covered by the tile ranges of the last sort
    int rest_n[kMaxSpecies];   // entries on the rest list of the last tile launch
    double red[4];
    unsigned long long live;
    unsigned long long contmax;
    unsigned int jmax;
    int pad1;
};

// Largest sort key space of any tiling with tiles of at most kMaxTile cells
// per axis (ragged last tiles pad the key space up to a whole tile).
constexpr int kMaxTile = 16;
// Smallest tile edge (keeps the per-species tile ranges small).
constexpr int kMinTile = 3;

int64_t max_keys(const pic_grid_desc* d) {
    int64_t k = 1;
    for (int a = 0; a < 3; ++a) k *= (int64_t)d->n[a] + kMaxTile - 1;
    return k;
}

// Most tiles any accepted tiling can have.
int64_t max_tiles(const pic_grid_desc* d) {
    int64_t k = 1;
    for (int a = 0; a < 3; ++a) k *= ((int64_t)d->n[a] + kMinTile - 1) / kMinTile;
    return k;
}

// nullptr if the tiling is acceptable for a grid of n cells, else the reason.
const char* validate_tiling(const int32_t n[3], const int32_t tile[3], int32_t guard, int32_t threads,
                            int32_t interleave, int32_t sort_interval) {
    for (int a = 0; a < 3; ++a) {
        if (tile[a] < 0 || (tile[a] > 0 && tile[a] > n[a])) return "tile larger than the grid";
        if (tile[a] > kMaxTile) return "tile above 16 cells per axis";
        if (tile[a] > 0 && tile[a] < kMinTile) return "tile below 3 cells per axis";
    }
    if (sort_interval < 0) return "negative sort interval";
    if (guard > 3) return "tile guard above 3 cells";
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return "threads per tile must be 256, 512 or 1024";
    if (interleave < 0) return "negative interleave";
    pic_grid_desc tmp{};
    for (int a = 0; a < 3; ++a) {
        tmp.n[a] = n[a];
        tmp.tile[a] = tile[a];
    }
    tmp.guard = guard;
    const Tiling tl = tiling_of(&tmp);
    if (tile_lds_bytes(tl.t, tl.guard) > kMaxLds) return "tile and guard exceed the 160 KiB of LDS";
    return nullptr;
}

Layout layout(const pic_grid_desc* d, int64_t maxp) {
    const int64_t ncell = (int64_t)d->n[0] * d->n[1] * d->n[2];
    const int64_t nkeys = max_keys(d);
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.acc = take(3 * (size_t)ncell * 8);
    L.jtmp = take(3 * (size_t)ncell * 4);
    L.rho = take((size_t)ncell * 8);
    L.small = take(sizeof(Small));
    L.prev_cell = take((size_t)maxp * 4);
    L.prev_off = take(3 * align_up((size_t)maxp * 4));
    L.alt_cell = take((size_t)maxp * 4);
    L.alt_off = take(3 * align_up((size_t)maxp * 4));
    L.alt_u = take(3 * align_up((size_t)maxp * 4));
    L.alt_w = take((size_t)maxp * 4);
    L.alt_id = take((size_t)maxp * 4);
    L.sort_rank = take((size_t)maxp * 4);
    L.hist = take(((size_t)nkeys + 1) * 4);
    L.sort_lc = take((size_t)nkeys * 4);
    L.sums = take((((size_t)nkeys + 1 + 1023) / 1024 + 1) * 4);
    L.toff_stride = align_up(((size_t)max_tiles(d) + 1) * 4);
    L.toff = take(kMaxSpecies * L.toff_stride);
    const bool dn = d->jpost == PIC_JPOST_DENOISER;
    L.dn_w = take(dn ? (kDnW1 + kDnW2 + kDnW3) * 2 + kDnBias * 4 : 0);
    L.dn_h1 = take(dn ? (size_t)ncell * 64 : 0);
    L.dn_h2 = take(dn ? (size_t)ncell * 64 : 0);
    // run diagnostics: spectrum bins (charge, count), reduction words, axis line
    L.diag = take(kDiagBytesFixed + (size_t)d->n[0] * 8);
    L.total = o;
    return L;
}

struct Species {
    pic_species_bufs user;   // caller's arrays
    pic_species_bufs cur;    // arrays holding the current data (user's or the workspace copy)
    pic_species_bufs alt;    // the other set
    int64_t base;            // offset into per-particle workspace arrays
    int64_t bound;           // host upper bound of the particle count
    int64_t sort_step;       // step of the last sort
    bool sorted;             // tile ranges valid
    bool prev_valid;         // x^n of the last split gather_push kept
};

// Phase timing: an event recorded before and after each timed phase.
enum { PH_SORT, PH_TILE, PH_LOOSE, PH_JPOST, PH_FIELD, PH_WINDOW, PH_COUNT };

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Mark {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    int64_t steps = 0, sorts = 0, tiles = 0;
    ~Prof() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
    // record an event (nullptr when timing is off)
    hipError_t mark(hipStream_t st, hipEvent_t* ev) {
        *ev = nullptr;
        if (!on) return hipSuccess;
        if (used == pool.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            pool.push_back(e);
        }
        *ev = pool[used++];
        return hipEventRecord(*ev, st);
    }
    hipError_t end(hipStream_t st, int phase, hipEvent_t start) {
        if (!on || !start) return hipSuccess;
        hipEvent_t e;
        hipError_t r = mark(st, &e);
        if (r != hipSuccess) return r;
        marks.push_back({phase, start, e});
        return hipSuccess;
    }
    hipError_t enable(hipStream_t st, bool en) {
        if (en) {
            hipError_t r = hipStreamSynchronize(st);
            if (r != hipSuccess) return r;
            marks.clear();
            used = 0;
            steps = sorts = tiles = 0;
        }
        on = en;
        return hipSuccess;
    }
    hipError_t read(hipStream_t st, pic_profile* out) {
        hipError_t r = hipStreamSynchronize(st);
        if (r != hipSuccess) return r;
        double ms[PH_COUNT] = {0, 0, 0, 0, 0, 0};
        for (const auto& m : marks) {
            float t = 0.0f;
            r = hipEventElapsedTime(&t, m.a, m.b);
            if (r != hipSuccess) return r;
            ms[m.phase] += t;
        }
        out->sort_ms = ms[PH_SORT];
        out->tile_ms = ms[PH_TILE];
        out->loose_ms = ms[PH_LOOSE];
        out->jpost_ms = ms[PH_JPOST];
        out->field_ms = ms[PH_FIELD];
        out->window_ms = ms[PH_WINDOW];
        out->steps = steps;
        out->sorts = sorts;
        out->tile_launches = tiles;
        return hipSuccess;
    }
};

}  // namespace

struct pic_ctx {
    pic_grid_desc desc;
    pic_field_bufs f;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    int64_t maxp;
    int64_t pused;
    Layout L;
    Tiling tl;
    Geom g;
    PDCoef pd;
    std::vector<Species> sp;
    int64_t step;
    std::string err;
    // laser source and moving window
    bool has_laser = false;
    pic_laser_desc laser;
    int64_t window_start = INT64_MAX;
    int64_t shift = 0;
    bool has_plasma[kMaxSpecies] = {};
    PlasmaDev plasma[kMaxSpecies];
    // learned current denoiser (pic_denoiser_set)
    bool has_dn = false;
    DenoiseWeights dn{};
    // phase timing (pic_profile_*)
    Prof prof;
    // a split-path step is in progress (pic_gather_push since the last pic_field_step)
    bool mid_step = false;
    // the J planes hold the post-processed current (binomial or denoiser
    // output) rather than the raw deposit: the continuity check filters rho
    bool j_filtered = false;
    // transverse absorbing layer (pic_set_pml); g.pml holds its thickness
    pic_pml_desc pml_desc{};
    PmlDev pml{};
    char* pml_buf = nullptr;
    size_t pml_state_bytes = 0;   // the auxiliary arrays (checkpointed), after the coefficient table
};

namespace {

pic_status fail(pic_ctx* c, pic_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define HIPCHK(ctx, expr)                                                                           \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(ctx, PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define PICCHK(expr)                      \
    do {                                  \
        pic_status s_ = (expr);           \
        if (s_ != PIC_OK) return s_;      \
    } while (0)

pic_status validate(const pic_grid_desc* d, char* msg, size_t len) {
    auto bad = [&](const char* why) {
        if (msg && len) snprintf(msg, len, "%s", why);
        return PIC_EINVAL;
    };
    if (!d) return bad("null descriptor");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 4) return bad("every axis needs at least 4 cells");
        if (!(d->d[a] > 0.0) || !isfinite(d->d[a])) return bad("cell sizes must be positive and finite");
    }
    if ((int64_t)d->n[0] * d->n[1] * d->n[2] >= (1ll << 31)) return bad("grid exceeds 2^31 cells");
    if (!(d->dt > 0.0) || !isfinite(d->dt)) return bad("dt must be positive and finite");
    if (d->solver != PIC_SOLVER_YEE && d->solver != PIC_SOLVER_PD) return bad("unknown solver");
    if (d->bc_x != PIC_BC_PERIODIC && d->bc_x != PIC_BC_MOVING_WINDOW) return bad("unknown x boundary");
    if (d->jpost < PIC_JPOST_NONE || d->jpost > PIC_JPOST_DENOISER) return bad("unknown current post-processing");
    if (d->pd_variant < 0 || d->pd_variant > 1) return bad("unknown perfect-dispersion variant");
    if (max_keys(d) >= (1ll << 31)) return bad("tile key space exceeds 2^31");
    const char* why = validate_tiling(d->n, d->tile, d->guard, d->threads, d->interleave, d->sort_interval);
    if (why) return bad(why);
    if (d->solver == PIC_SOLVER_YEE) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += 1.0 / (d->d[a] * d->d[a]);
        if (!(d->dt < 1.0 / sqrt(s))) return bad("Yee time step violates the Courant limit");
    } else {
        if (d->d[0] > d->d[1] || d->d[0] > d->d[2])
            return bad("perfect dispersion requires dx <= dy and dx <= dz");
        if (d->dt > d->d[0] * (1.0 + 1e-12)) return bad("perfect dispersion requires c dt <= dx");
    }
    if (d->bc_x == PIC_BC_MOVING_WINDOW && d->n[0] < 2 * kKillMargin + 4)
        return bad("moving window needs at least 10 cells along x");
    if (msg && len) msg[0] = 0;
    return PIC_OK;
}

// Transverse smoothing coefficients of the perfect-dispersion curl.  With
// r_y = (dx/dy)^2 and r_z = (dx/dz)^2: beta = (1/8, r_y/8, r_z/8), corner
// weights gamma_yz = r_y r_z/16, gamma_zx = r_z/16, gamma_xy = r_y/16 (zero for
// variant 1), centres alpha_d = 1 - 2 beta_t1 - 2 beta_t2 - 4 gamma_{t1t2}.
void pd_coefficients(const pic_grid_desc* d, PDCoef* c) {
    if (d->solver != PIC_SOLVER_PD) {
        for (int a = 0; a < 3; ++a) {
            c->alpha[a] = 1.0f;
            c->beta[a] = 0.0f;
            c->gam[a] = 0.0f;
        }
        return;
    }
    const double ry = (d->d[0] / d->d[1]) * (d->d[0] / d->d[1]);
    const double rz = (d->d[0] / d->d[2]) * (d->d[0] / d->d[2]);
    const double beta[3] = {0.125, 0.125 * ry, 0.125 * rz};
    double gam[3] = {ry * rz / 16.0, rz / 16.0, ry / 16.0};
    if (d->pd_variant == 1) gam[0] = gam[1] = gam[2] = 0.0;
    for (int a = 0; a < 3; ++a) {
        const int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
        c->alpha[a] = (float)(1.0 - 2.0 * beta[t1] - 2.0 * beta[t2] - 4.0 * gam[a]);
        c->beta[a] = (float)beta[a];
        c->gam[a] = (float)gam[a];
    }
}

Small* small_of(pic_ctx* c) { return reinterpret_cast<Small*>(c->ws + c->L.small); }

SpeciesDev dev_from(const pic_ctx* c, const Species& s, const pic_species_bufs& b) {
    SpeciesDev d;
    d.cell = b.cell;
    for (int a = 0; a < 3; ++a) {
        d.off[a] = b.off[a];
        d.u[a] = b.u[a];
    }
    d.w = b.w;
    d.id = b.id;
    d.qmh = (float)(s.user.q * c->desc.dt / (2.0 * s.user.m));
    d.mq = (float)(-s.user.q);
    return d;
}

SpeciesDev dev_of(const pic_ctx* c, const Species& s) { return dev_from(c, s, s.cur); }

PrevDev prev_of(pic_ctx* c, const Species& s) {
    PrevDev p;
    p.cell = reinterpret_cast<int*>(c->ws + c->L.prev_cell) + s.base;
    const size_t stride = align_up((size_t)c->maxp * 4);
    for (int a = 0; a < 3; ++a) p.off[a] = reinterpret_cast<float*>(c->ws + c->L.prev_off + a * stride) + s.base;
    return p;
}

FieldPtrs fields_of(pic_ctx* c) {
    FieldPtrs f;
    for (int a = 0; a < 3; ++a) {
        f.E[a] = c->f.E[a];
        f.B[a] = c->f.B[a];
    }
    return f;
}

unsigned long long* acc_of(pic_ctx* c) { return reinterpret_cast<unsigned long long*>(c->ws + c->L.acc); }
int* hist_of(pic_ctx* c) { return reinterpret_cast<int*>(c->ws + c->L.hist); }
// The level-order sort's scratch (one int per particle slot of the species):
// the split path's saved positions, which every sort invalidates anyway.
int* level_of(pic_ctx* c, const Species& sp) { return reinterpret_cast<int*>(c->ws + c->L.prev_cell) + sp.base; }
int* toff_of(pic_ctx* c, int32_t s) { return reinterpret_cast<int*>(c->ws + c->L.toff + (size_t)s * c->L.toff_stride); }

void jtmp_of(pic_ctx* c, float* out[3]) {
    for (int a = 0; a < 3; ++a) out[a] = reinterpret_cast<float*>(c->ws + c->L.jtmp) + (size_t)a * c->g.ncell;
}

void jscale(const pic_ctx* c, double s[3]) {
    for (int a = 0; a < 3; ++a) s[a] = PIC_FIX_INV * c->desc.d[a] / c->desc.dt;
}

pic_status check_species(pic_ctx* c, int32_t s) {
    if (!c) return PIC_EINVAL;
    if (s < 0 || s >= (int32_t)c->sp.size()) return fail(c, PIC_EINVAL, "no species %d", s);
    return PIC_OK;
}

// Read and clear the device error flags; map them to a status.
pic_status device_errors(pic_ctx* c) {
    int flags = 0;
    HIPCHK(c, hipMemcpyAsync(&flags, &small_of(c)->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flags) {
        HIPCHK(c, hipMemsetAsync(&small_of(c)->err, 0, sizeof(int), c->stream));
        if (flags & ERR_NONFINITE) return fail(c, PIC_ENONFINITE, "non-finite momentum on the device");
        if (flags & ERR_CFL) return fail(c, PIC_ECFL, "a particle moved one cell or more in a step");
        if (flags & ERR_OVERFLOW) return fail(c, PIC_EOVERFLOW, "invalid cell index or capacity overflow on the device");
    }
    return PIC_OK;
}

// Incident laser field on the source plane: e(t) = -d/dt [a0 env(t) cos(w0 (t - t_peak))],
// env = exp(-2 ln2 (t - t_peak)^2 / fwhm^2).
double laser_e(const pic_laser_desc& L, double t) {
    const double tau = t - L.t_peak;
    const double k = 2.0 * log(2.0) / (L.fwhm * L.fwhm);
    const double env = exp(-k * tau * tau);
    const double denv = -2.0 * k * tau * env;
    const double ph = L.omega0 * tau;
    return L.a0 * (env * L.omega0 * sin(ph) - denv * cos(ph));
}

// Total-field/scattered-field correction of one field plane: B_z behind the
// source gets + h e(t) f / dx, E_y on the source gets + dt e(t + dx/2) f / dx.
pic_status laser_plane(pic_ctx* c, bool e_plane, double h, double t) {
    const pic_laser_desc& L = c->laser;
    const double amp = e_plane ? laser_e(L, t + 0.5 * c->desc.d[0]) : laser_e(L, t);
    const int ix = e_plane ? L.src_x : L.src_x - 1;
    float* F = e_plane ? c->f.E[1] : c->f.B[2];
    HIPCHK(c, launch_laser_plane(c->g, F, ix, h * amp / c->desc.d[0], L.yc, L.zc, L.waist, c->desc.d[1],
                                 c->desc.d[2], c->stream));
    return PIC_OK;
}

// Field update of the step that starts at t = step dt: B half step, E step,
// B half step (Section 2, eq. 2.1), with the laser source while it is active.
pic_status field_update(pic_ctx* c, float* const Juse[3]) {
    FieldPtrs f = fields_of(c);
    const int pd = c->desc.solver == PIC_SOLVER_PD;
    const double dt = c->desc.dt, t = c->step * dt;
    const bool laser = c->has_laser && c->shift == 0 && t <= c->laser.t_end;
    const PmlDev* pml = c->g.pml ? &c->pml : nullptr;
    HIPCHK(c, launch_bhalf(c->g, pd, c->pd, f.E, f.B, (float)(0.5 * dt), pml, 1, c->stream));
    if (laser) PICCHK(laser_plane(c, false, 0.5 * dt, t));
    HIPCHK(c, launch_efull(c->g, f.E, f.B, Juse, pml, c->stream));
    if (laser) PICCHK(laser_plane(c, true, dt, t + 0.5 * dt));
    HIPCHK(c, launch_bhalf(c->g, pd, c->pd, f.E, f.B, (float)(0.5 * dt), pml, 0, c->stream));
    if (laser) PICCHK(laser_plane(c, false, 0.5 * dt, t + dt));
    return PIC_OK;
}

// Exact particle count of a species (synchronises); refreshes the host bounds.
pic_status refresh_bound(pic_ctx* c, int32_t s) {
    int v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, &small_of(c)->count[s], sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->sp[s].bound = v;
    return PIC_OK;
}

pic_status inject_slab(pic_ctx* c, int32_t s, int32_t xb, int32_t xe) {
    Species& sp = c->sp[s];
    const PlasmaDev& P = c->plasma[s];
    const int64_t most = (int64_t)(xe - xb) * c->g.n[1] * c->g.n[2] * P.ppc[0] * P.ppc[1] * P.ppc[2];
    if (most <= 0) return PIC_OK;
    if (sp.bound + most > sp.user.capacity) {
        PICCHK(refresh_bound(c, s));
        if (sp.bound + most > sp.user.capacity)
            return fail(c, PIC_ENOMEM, "species %d: %lld particles plus up to %lld injected exceed capacity %lld", s,
                        (long long)sp.bound, (long long)most, (long long)sp.user.capacity);
    }
    HIPCHK(c, launch_inject(c->g, P, dev_of(c, sp), (long long)c->shift, xb, xe, &small_of(c)->count[s],
                            (int)sp.user.capacity, &small_of(c)->err, c->stream));
    sp.bound += most;
    return PIC_OK;
}

pic_status prof_mark(pic_ctx* c, hipEvent_t* ev) {
    HIPCHK(c, c->prof.mark(c->stream, ev));
    return PIC_OK;
}

pic_status prof_end(pic_ctx* c, int phase, hipEvent_t start) {
    HIPCHK(c, c->prof.end(c->stream, phase, start));
    return PIC_OK;
}

// End of a step: count it; move the window one cell when it is due.
pic_status end_step(pic_ctx* c) {
    c->step += 1;
    if (c->prof.on) c->prof.steps += 1;
    if (!c->g.window || c->step < c->window_start) return PIC_OK;
    hipEvent_t t0;
    PICCHK(prof_mark(c, &t0));
    HIPCHK(c, launch_clear_plane(c->g, fields_of(c), c->g.origin, c->stream));
    if (c->g.pml) HIPCHK(c, launch_clear_pml_plane(c->g, c->pml, c->g.origin, c->stream));
    c->g.origin = c->g.origin + 1 == c->g.n[0] ? 0 : c->g.origin + 1;
    c->shift += 1;
    const int slab = c->g.n[0] - 1 - c->g.kill_hi;
    for (int32_t s = 0; s < (int32_t)c->sp.size(); ++s)
        if (c->has_plasma[s]) PICCHK(inject_slab(c, s, slab, slab + 1));
    return prof_end(c, PH_WINDOW, t0);
}

// copy = false: the particle data stay in the pre-sort set (now sp.alt) and
// the tile step that must follow gathers them (launch_pic_tile with src).
pic_status sort_species(pic_ctx* c, int32_t s, bool copy) {
    Species& sp = c->sp[s];
    Small* sm = small_of(c);
    int* rank = reinterpret_cast<int*>(c->ws + c->L.sort_rank) + sp.base;
    HIPCHK(c, launch_sort(c->g, c->tl.t, dev_from(c, sp, sp.cur), dev_from(c, sp, sp.alt), &sm->count[s],
                          &sm->sorted[s], (int)sp.bound, hist_of(c), rank, reinterpret_cast<int*>(c->ws + c->L.sums),
                          level_of(c, sp), reinterpret_cast<int*>(c->ws + c->L.sort_lc), c->tl.interleave,
                          toff_of(c, s), copy, sp.sorted, c->stream));
    std::swap(sp.cur, sp.alt);
    sp.sorted = true;
    sp.sort_step = c->step;
    sp.prev_valid = false;
    return PIC_OK;
}

// Boundary rule of the denoiser's convolutions for this grid.
void dn_bc(const pic_ctx* c, int bc[3]) {
    bc[0] = c->g.window ? 2 : 0;
    bc[1] = 0;
    bc[2] = 0;
}

// Jin -> Jout through the denoiser (distinct buffers).
pic_status denoise(pic_ctx* c, float* const Jin[3], float* const Jout[3]) {
    if (!c->has_dn) return fail(c, PIC_ESTATE, "denoiser weights not set");
    int bc[3];
    dn_bc(c, bc);
    HIPCHK(c, launch_denoise(c->g, bc, c->dn, Jin, Jout, reinterpret_cast<__bf16*>(c->ws + c->L.dn_h1),
                             reinterpret_cast<__bf16*>(c->ws + c->L.dn_h2), c->stream));
    return PIC_OK;
}

// J post-processing in place (through the workspace current).
pic_status filter_in_place(pic_ctx* c) {
    if (c->desc.jpost == PIC_JPOST_NONE) return PIC_OK;
    float* tmp[3];
    jtmp_of(c, tmp);
    if (c->desc.jpost == PIC_JPOST_BINOMIAL)
        HIPCHK(c, launch_binomial(c->g, c->f.J, tmp, c->stream));
    else
        PICCHK(denoise(c, c->f.J, tmp));
    for (int a = 0; a < 3; ++a)
        HIPCHK(c, hipMemcpyAsync(c->f.J[a], tmp[a], (size_t)c->g.ncell * 4, hipMemcpyDeviceToDevice, c->stream));
    c->j_filtered = true;
    return PIC_OK;
}

// Current post-processing and field update of one production step.
pic_status finish_step(pic_ctx* c) {
    double sc[3];
    jscale(c, sc);
    float* Juse[3] = {c->f.J[0], c->f.J[1], c->f.J[2]};
    hipEvent_t t0, t1;
    PICCHK(prof_mark(c, &t0));
    if (c->desc.jpost == PIC_JPOST_BINOMIAL) {
        float* tmp[3];
        jtmp_of(c, tmp);
        HIPCHK(c, launch_jfinal(c->g, acc_of(c), tmp, sc, 1, c->stream));
        HIPCHK(c, launch_binomial(c->g, tmp, c->f.J, c->stream));
    } else if (c->desc.jpost == PIC_JPOST_NONE) {
        HIPCHK(c, launch_jfinal(c->g, acc_of(c), c->f.J, sc, 1, c->stream));
    } else {
        float* tmp[3];
        jtmp_of(c, tmp);
        HIPCHK(c, launch_jfinal(c->g, acc_of(c), tmp, sc, 1, c->stream));
        PICCHK(denoise(c, tmp, c->f.J));
    }
    c->j_filtered = c->desc.jpost != PIC_JPOST_NONE;
    PICCHK(prof_end(c, PH_JPOST, t0));
    PICCHK(prof_mark(c, &t1));
    PICCHK(field_update(c, Juse));
    PICCHK(prof_end(c, PH_FIELD, t1));
    return end_step(c);
}


// ---- transverse absorbing layer -----------------------------------------------
// Buffer: the coefficient table (16 L floats), then y[0..3] (n[0] 2L n[2]
// floats each), then z[0..3] (n[0] n[1] 2L each), every part 256-byte aligned.
struct PmlLayout {
    size_t coef, y[4], z[4], total;
};

bool pml_layout(const pic_grid_desc* d, const pic_pml_desc* p, PmlLayout* out) {
    if (!d || !p || validate(d, nullptr, 0) != PIC_OK) return false;
    const int L = p->layers;
    if (L < 8 || 2 * L + 1 > d->n[1] || 2 * L + 1 > d->n[2]) return false;
    auto up = [](size_t b) { return (b + kAlign - 1) / kAlign * kAlign; };
    size_t o = 0;
    out->coef = o;
    o += up((size_t)16 * L * 4);
    const size_t ny = (size_t)d->n[0] * 2 * L * d->n[2] * 4, nz = (size_t)d->n[0] * d->n[1] * 2 * L * 4;
    for (int a = 0; a < 4; ++a) {
        out->y[a] = o;
        o += up(ny);
    }
    for (int a = 0; a < 4; ++a) {
        out->z[a] = o;
        o += up(nz);
    }
    out->total = o;
    return true;
}

// sigma at position p (cells) along an axis of n cells with a layer of L cells
double pml_sigma_at(double smax, double grade, int L, int n, double p) {
    const double lo = (L - 1.0 - p) / L, hi = (p - (double)(n - L)) / L;
    double depth = std::max(lo, hi);
    if (!(depth > 0.0)) return 0.0;
    depth = std::min(depth, 1.0);
    return smax * pow(depth, grade);
}

// ---- checkpoint blob ---------------------------------------------------------
// header, then E[3], B[3], J[3] (ncell floats each), then per species its
// `count` particles as cell, off[3], u[3], w, id arrays (4 bytes per value).
constexpr uint64_t kCkptMagic = 0x4b43353533434950ull;   // "PIC355CK" little-endian
constexpr uint32_t kCkptVersion = 2;

struct CkptHeader {
    uint64_t magic;
    uint32_t version;
    uint32_t nspecies;
    int32_t n[3];
    int32_t origin;
    int32_t solver, bc_x;
    int32_t pml_layers;
    int32_t pad_;
    double d[3];
    double dt;
    int64_t step;
    int64_t shift;
    int64_t count[kMaxSpecies];
};

constexpr int kCkptArrays = 9;   // cell, off[3], u[3], w, id

size_t ckpt_bytes(const pic_ctx* c, const int64_t* count) {
    size_t b = sizeof(CkptHeader) + 9 * (size_t)c->g.ncell * 4 + (c->g.pml ? c->pml_state_bytes : 0);
    for (size_t s = 0; s < c->sp.size(); ++s) b += (size_t)count[s] * 4 * kCkptArrays;
    return b;
}

// The nine per-particle arrays of a buffer set, in blob order.
void ckpt_arrays(const pic_species_bufs& b, void* out[kCkptArrays]) {
    out[0] = b.cell;
    for (int a = 0; a < 3; ++a) {
        out[1 + a] = b.off[a];
        out[4 + a] = b.u[a];
    }
    out[7] = b.w;
    out[8] = b.id;
}

// Exact particle counts of every species (synchronises).
pic_status exact_counts(pic_ctx* c, int64_t* count) {
    int cnt[kMaxSpecies] = {};
    HIPCHK(c, hipMemcpyAsync(cnt, small_of(c)->count, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    PICCHK(device_errors(c));
    for (size_t s = 0; s < c->sp.size(); ++s) count[s] = cnt[s];
    return PIC_OK;
}

}  // namespace

// ---- batched launcher ------------------------------------------------------

struct pic_batch {
    std::vector<pic_ctx*> m;
    int nsp = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t tab_bytes = 0;    // member table of one slot
    size_t slot_bytes = 0;   // table + flat tile offsets
    char* host = nullptr;    // pinned staging ring (nslots slots)
    std::vector<hipEvent_t> ev;
    std::vector<bool> used;
    int next = 0;
    std::string err;
    Prof prof;
    ~pic_batch() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        if (host) (void)hipHostFree(host);
    }
};

namespace {

constexpr int kBatchSlots = 16;

size_t batch_tab_bytes(int32_t n) { return align_up((size_t)n * sizeof(InstDesc)); }
size_t batch_slot_bytes(int32_t n) { return batch_tab_bytes(n) + align_up(((size_t)n + 1) * sizeof(int)); }

pic_status bfail(pic_batch* b, pic_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
    return st;
}

#define BHIPCHK(b, expr)                                                                             \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return bfail(b, PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// Member status -> batch error naming the member.
pic_status bmember(pic_batch* b, int i, pic_status st) {
    if (st != PIC_OK) bfail(b, st, "member %d: %s", i, b->m[i]->err.c_str());
    return st;
}

// Descriptor of member c for species s at the start of its current step.
void fill_desc(pic_ctx* c, int32_t s, InstDesc& d) {
    Species& sp = c->sp[s];
    memset(&d, 0, sizeof d);
    d.g = c->g;
    d.t = c->tl.t;
    d.guard = c->tl.guard;
    d.pd = c->desc.solver == PIC_SOLVER_PD;
    d.depth = c->tl.interleave;
    d.nkeys = c->tl.t.ntiles * c->tl.t.tcells;
    d.sdiv = make_sortdiv(c->g, c->tl.t);
    d.c = c->pd;
    d.f = fields_of(c);
    float* jt[3];
    jtmp_of(c, jt);
    for (int a = 0; a < 3; ++a) {
        d.J[a] = c->f.J[a];
        d.Jt[a] = jt[a];
    }
    d.jpost = c->desc.jpost == PIC_JPOST_BINOMIAL;
    d.sorting = !sp.sorted || c->step - sp.sort_step >= c->tl.sort_interval;
    d.s = dev_from(c, sp, sp.cur);
    d.alt = dev_from(c, sp, sp.alt);
    d.hist = hist_of(c);
    d.toff = toff_of(c, s);
    d.rank = reinterpret_cast<int*>(c->ws + c->L.sort_rank) + sp.base;
    d.sums = reinterpret_cast<int*>(c->ws + c->L.sums);
    d.level = level_of(c, sp);
    d.lc = reinterpret_cast<int*>(c->ws + c->L.sort_lc);
    d.resort = d.sorting && sp.sorted;   // (the batch step marks the species sorted after this)
    d.acc = acc_of(c);
    Small* sm = small_of(c);
    d.err = &sm->err;
    d.count = &sm->count[s];
    d.sorted = &sm->sorted[s];
    d.rest_n = &sm->rest_n[s];
    d.capacity = (int)sp.user.capacity;
    d.hdt = (float)(0.5 * c->desc.dt);
    jscale(c, d.jscale);
    // laser planes, with the same arithmetic as field_update / laser_plane
    const double dt = c->desc.dt, t = c->step * dt;
    d.laser_on = c->has_laser && c->shift == 0 && t <= c->laser.t_end;
    if (d.laser_on) {
        const pic_laser_desc& L = c->laser;
        const double dx = c->desc.d[0];
        const double h = 0.5 * dt;
        d.lcoef[0] = h * laser_e(L, t) / dx;
        d.lcoef[1] = dt * laser_e(L, (t + 0.5 * dt) + 0.5 * dx) / dx;
        d.lcoef[2] = h * laser_e(L, t + dt) / dx;
        d.lix_b = L.src_x - 1;
        d.lix_e = L.src_x;
        d.yc = L.yc;
        d.zc = L.zc;
        d.inv_w2 = 1.0 / (L.waist * L.waist);
        d.dy = c->desc.d[1];
        d.dz = c->desc.d[2];
    }
    d.wmove = c->g.window && c->step + 1 >= c->window_start;
    d.inject = d.wmove && c->has_plasma[s];
    d.slab = c->g.n[0] - 1 - c->g.kill_hi;
    d.shift = c->shift + (d.wmove ? 1 : 0);
    if (c->has_plasma[s]) d.plasma = c->plasma[s];
}

// Stage the member table (and flat tile offsets) of species s into the next
// ring slot; returns the device addresses.
pic_status upload_tables(pic_batch* b, int32_t s, InstDesc** dtab, int** dbegin, int* total_tiles) {
    const int n = (int)b->m.size();
    const int k = b->next;
    b->next = (k + 1) % kBatchSlots;
    if (b->used[k]) BHIPCHK(b, hipEventSynchronize(b->ev[k]));
    char* h = b->host + (size_t)k * b->slot_bytes;
    InstDesc* tab = reinterpret_cast<InstDesc*>(h);
    int* begin = reinterpret_cast<int*>(h + b->tab_bytes);
    int64_t tot = 0;
    for (int i = 0; i < n; ++i) {
        fill_desc(b->m[i], s, tab[i]);
        begin[i] = (int)tot;
        tot += b->m[i]->tl.t.ntiles;
    }
    if (tot >= (1ll << 31)) return bfail(b, PIC_EINVAL, "more than 2^31 tiles in the batch");
    begin[n] = (int)tot;
    char* dslot = b->ws + (size_t)k * b->slot_bytes;
    BHIPCHK(b, hipMemcpyAsync(dslot, h, b->slot_bytes, hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipEventRecord(b->ev[k], b->stream));
    b->used[k] = true;
    *dtab = reinterpret_cast<InstDesc*>(dslot);
    *dbegin = reinterpret_cast<int*>(dslot + b->tab_bytes);
    *total_tiles = (int)tot;
    return PIC_OK;
}

pic_status bmark(pic_batch* b, hipEvent_t* e) {
    BHIPCHK(b, b->prof.mark(b->stream, e));
    return PIC_OK;
}

pic_status bend(pic_batch* b, int phase, hipEvent_t e) {
    BHIPCHK(b, b->prof.end(b->stream, phase, e));
    return PIC_OK;
}

// One step of every member: per species sort (members due), tiled step and
// rest pass; then current read-out, field update with laser planes and
// window motion with injection.  The host bookkeeping mirrors pic_step.
pic_status batch_one_step(pic_batch* b) {
    const int n = (int)b->m.size();
    InstDesc* dtab = nullptr;
    int* dbegin = nullptr;
    for (int32_t s = 0; s < b->nsp; ++s) {
        int total = 0;
        PICCHK(upload_tables(b, s, &dtab, &dbegin, &total));
        int max_sort = 0, max_keys1 = 0, max_tiles1 = 0, max_tcells = 1;
        bool any_sort = false, all_888g1 = true;
        size_t lds = 0;
        for (int i = 0; i < n; ++i) {
            pic_ctx* c = b->m[i];
            Species& sp = c->sp[s];
            const bool sorting = !sp.sorted || c->step - sp.sort_step >= c->tl.sort_interval;
            if (sorting) {
                any_sort = true;
                max_sort = (int)std::max<int64_t>(max_sort, sp.bound);
                max_keys1 = std::max(max_keys1, c->tl.t.ntiles * c->tl.t.tcells + 1);
                max_tiles1 = std::max(max_tiles1, c->tl.t.ntiles + 1);
                max_tcells = std::max(max_tcells, c->tl.t.tcells);
                std::swap(sp.cur, sp.alt);
                sp.sorted = true;
                sp.sort_step = c->step;
            }
            sp.prev_valid = false;
            lds = std::max(lds, tile_lds_bytes(c->tl.t, c->tl.guard));
            all_888g1 = all_888g1 && c->tl.t.T[0] == 8 && c->tl.t.T[1] == 8 && c->tl.t.T[2] == 8 && c->tl.guard == 1;
        }
        hipEvent_t t0, t1, t2;
        if (any_sort) {
            PICCHK(bmark(b, &t0));
            BHIPCHK(b, launch_batch_sort(dtab, n, max_sort, max_keys1, max_tiles1, max_tcells, b->stream));
            PICCHK(bend(b, PH_SORT, t0));
            if (b->prof.on) b->prof.sorts += 1;
        }
        PICCHK(bmark(b, &t1));
        BHIPCHK(b, launch_batch_tile(dtab, dbegin, n, total, b->m[0]->tl.threads, lds, all_888g1, b->stream));
        PICCHK(bend(b, PH_TILE, t1));
        if (b->prof.on) b->prof.tiles += 1;
        PICCHK(bmark(b, &t2));
        BHIPCHK(b, launch_batch_rest(dtab, n, b->stream));
        PICCHK(bend(b, PH_LOOSE, t2));
        // the window phase below needs each species' table; keep species 0's
        // for the field phase and re-stage the others then
    }
    // current read-out and field update (member-wide parts of the last table)
    int max_cells = 0, max_plane = 0, max_btiles = 0;
    bool any_bin = false, any_laser = false, any_move = false;
    for (int i = 0; i < n; ++i) {
        pic_ctx* c = b->m[i];
        max_cells = std::max(max_cells, c->g.ncell);
        max_btiles = std::max(max_btiles, bhalf_tiles(c->g.n));
        max_plane = std::max(max_plane, c->g.n[1] * c->g.n[2]);
        any_bin = any_bin || c->desc.jpost == PIC_JPOST_BINOMIAL;
        const double t = c->step * c->desc.dt;
        any_laser = any_laser || (c->has_laser && c->shift == 0 && t <= c->laser.t_end);
        any_move = any_move || (c->g.window && c->step + 1 >= c->window_start);
    }
    hipEvent_t t3, t4, t5;
    PICCHK(bmark(b, &t3));
    BHIPCHK(b, launch_batch_jfinal(dtab, n, max_cells, b->stream));
    if (any_bin) BHIPCHK(b, launch_batch_binomial(dtab, n, max_cells, b->stream));
    PICCHK(bend(b, PH_JPOST, t3));
    PICCHK(bmark(b, &t4));
    BHIPCHK(b, launch_batch_bhalf(dtab, n, max_btiles, b->stream));
    if (any_laser) BHIPCHK(b, launch_batch_laser(dtab, n, 0, max_plane, b->stream));
    BHIPCHK(b, launch_batch_efull(dtab, n, max_cells, b->stream));
    if (any_laser) BHIPCHK(b, launch_batch_laser(dtab, n, 1, max_plane, b->stream));
    BHIPCHK(b, launch_batch_bhalf(dtab, n, max_btiles, b->stream));
    if (any_laser) BHIPCHK(b, launch_batch_laser(dtab, n, 2, max_plane, b->stream));
    PICCHK(bend(b, PH_FIELD, t4));
    PICCHK(bmark(b, &t5));
    if (any_move) {
        BHIPCHK(b, launch_batch_clear(dtab, n, max_plane, b->stream));
        for (int32_t s = 0; s < b->nsp; ++s) {
            // capacity bound of the injected slab (exact count only when needed)
            long long max_cand = 0;
            bool any = false;
            for (int i = 0; i < n; ++i) {
                pic_ctx* c = b->m[i];
                if (!(c->g.window && c->step + 1 >= c->window_start) || !c->has_plasma[s]) continue;
                Species& sp = c->sp[s];
                const PlasmaDev& P = c->plasma[s];
                const int64_t most = (int64_t)c->g.n[1] * c->g.n[2] * P.ppc[0] * P.ppc[1] * P.ppc[2];
                if (sp.bound + most > sp.user.capacity) {
                    PICCHK(bmember(b, i, refresh_bound(c, s)));
                    if (sp.bound + most > sp.user.capacity)
                        return bfail(b, PIC_ENOMEM, "member %d species %d: %lld particles plus up to %lld injected exceed capacity %lld",
                                     i, s, (long long)sp.bound, (long long)most, (long long)sp.user.capacity);
                }
                sp.bound += most;
                max_cand = std::max<long long>(max_cand, most);
                any = true;
            }
            if (!any) continue;
            InstDesc* tab_s = dtab;
            if (s != b->nsp - 1) {
                int total = 0;
                int* dummy = nullptr;
                // the sort state of species s is already advanced: its arrays
                // are now `cur` with no sort pending
                PICCHK(upload_tables(b, s, &tab_s, &dummy, &total));
            }
            BHIPCHK(b, launch_batch_inject(tab_s, n, max_cand, b->stream));
        }
    }
    PICCHK(bend(b, PH_WINDOW, t5));
    // host bookkeeping of the step's end (end_step without the launches)
    for (int i = 0; i < n; ++i) {
        pic_ctx* c = b->m[i];
        const bool move = c->g.window && c->step + 1 >= c->window_start;
        c->step += 1;
        if (move) {
            c->g.origin = c->g.origin + 1 == c->g.n[0] ? 0 : c->g.origin + 1;
            c->shift += 1;
        }
    }
    if (b->prof.on) b->prof.steps += 1;
    return PIC_OK;
}

}  // namespace

// helpers of the run diagnostics
namespace {

double* diag_words(pic_ctx* c) {
    return reinterpret_cast<double*>(c->ws + c->L.diag) + 2 * kDiagBins;
}

// Bilinear weights of the transverse point (yc, zc) on component comp's grid.
void axis_weights(const pic_ctx* c, int comp, double yc, double zc, int* j0, int* k0, double* ty, double* tz) {
    static const double sy[6] = {0.0, 0.5, 0.0, 0.5, 0.0, 0.5};
    static const double sz[6] = {0.0, 0.0, 0.5, 0.5, 0.5, 0.0};
    const double gy = yc / c->desc.d[1] - sy[comp];
    const double gz = zc / c->desc.d[2] - sz[comp];
    const double fy = floor(gy), fz = floor(gz);
    *ty = gy - fy;
    *tz = gz - fz;
    // periodic y, z: bring the base node into [0, n)
    const long long jy = (long long)fy, kz = (long long)fz;
    *j0 = (int)(((jy % c->g.n[1]) + c->g.n[1]) % c->g.n[1]);
    *k0 = (int)(((kz % c->g.n[2]) + c->g.n[2]) % c->g.n[2]);
}

float* field_comp(pic_ctx* c, int comp) { return comp < 3 ? c->f.E[comp] : c->f.B[comp - 3]; }

}  // namespace

extern "C" {

size_t pic_workspace_bytes(const pic_grid_desc* desc, int64_t max_particles) {
    if (validate(desc, nullptr, 0) != PIC_OK || max_particles < 0) return 0;
    return layout(desc, max_particles > 0 ? max_particles : 1).total;
}

pic_status pic_validate_grid(const pic_grid_desc* desc, char* msg, size_t msg_len) {
    return validate(desc, msg, msg_len);
}

pic_status pic_init_grid(pic_ctx** out, const pic_grid_desc* desc, const pic_field_bufs* fields, void* workspace,
                         size_t workspace_bytes, int64_t max_particles, void* stream) {
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    char msg[256];
    pic_status st = validate(desc, msg, sizeof msg);
    if (st != PIC_OK) return st;
    if (!fields || !workspace || max_particles < 0) return PIC_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!fields->E[a] || !fields->B[a] || !fields->J[a]) return PIC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0) return PIC_EINVAL;
    const int64_t ncell = (int64_t)desc->n[0] * desc->n[1] * desc->n[2];
    const int64_t maxp = max_particles > 0 ? max_particles : 1;
    Layout L = layout(desc, maxp);
    if (workspace_bytes < L.total) return PIC_ENOMEM;
    pic_ctx* c = new (std::nothrow) pic_ctx();
    if (!c) return PIC_ENOMEM;
    c->desc = *desc;
    c->f = *fields;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    c->ws = reinterpret_cast<char*>(workspace);
    c->ws_bytes = workspace_bytes;
    c->maxp = maxp;
    c->pused = 0;
    c->L = L;
    c->tl = tiling_of(desc);
    c->step = 0;
    Geom& g = c->g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = desc->n[a];
        g.dtd[a] = (float)(desc->dt / desc->d[a]);
        g.inv_d[a] = (float)(1.0 / desc->d[a]);
    }
    g.nxy = desc->n[0] * desc->n[1];
    g.ncell = (int)ncell;
    g.window = desc->bc_x == PIC_BC_MOVING_WINDOW;
    g.origin = 0;
    g.kill_lo = kKillMargin;
    g.kill_hi = kKillMargin;
    g.dt = (float)desc->dt;
    pd_coefficients(desc, &c->pd);
    void* scratch_ptr = nullptr;   // this GPU's allocation-free scratch, looked up once per device
    hipError_t e = noalloc_scratch(&scratch_ptr);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.acc, 0, 3 * (size_t)ncell * 8, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.small, 0, sizeof(Small), c->stream);
    if (e != hipSuccess) {
        delete c;
        return PIC_EDEVICE;
    }
    *out = c;
    return PIC_OK;
}

pic_status pic_init_species(pic_ctx* c, const pic_species_bufs* bufs, int64_t n, int32_t* species_out) {
    if (!c || !bufs) return PIC_EINVAL;
    if ((int)c->sp.size() >= kMaxSpecies) return fail(c, PIC_EINVAL, "at most %d species", kMaxSpecies);
    if (!bufs->cell || !bufs->w || !bufs->id) return fail(c, PIC_EINVAL, "null particle array");
    for (int a = 0; a < 3; ++a)
        if (!bufs->off[a] || !bufs->u[a]) return fail(c, PIC_EINVAL, "null particle array");
    if (!(bufs->m > 0.0) || !isfinite(bufs->q)) return fail(c, PIC_EINVAL, "invalid charge or mass");
    if (n < 0 || n > bufs->capacity) return fail(c, PIC_EINVAL, "particle count outside [0, capacity]");
    if (bufs->capacity >= (1ll << 31)) return fail(c, PIC_EINVAL, "capacity exceeds 2^31");
    if (c->pused + bufs->capacity > c->maxp)
        return fail(c, PIC_ENOMEM, "workspace sized for %lld particles, species needs %lld more",
                    (long long)c->maxp, (long long)(c->pused + bufs->capacity - c->maxp));
    Species s;
    s.user = *bufs;
    s.cur = *bufs;
    s.base = c->pused;
    s.bound = n;
    s.sort_step = 0;
    s.sorted = false;
    s.prev_valid = false;
    const size_t stride = align_up((size_t)c->maxp * 4);
    s.alt = *bufs;
    s.alt.cell = reinterpret_cast<int32_t*>(c->ws + c->L.alt_cell) + s.base;
    for (int a = 0; a < 3; ++a) {
        s.alt.off[a] = reinterpret_cast<float*>(c->ws + c->L.alt_off + a * stride) + s.base;
        s.alt.u[a] = reinterpret_cast<float*>(c->ws + c->L.alt_u + a * stride) + s.base;
    }
    s.alt.w = reinterpret_cast<float*>(c->ws + c->L.alt_w) + s.base;
    s.alt.id = reinterpret_cast<int32_t*>(c->ws + c->L.alt_id) + s.base;
    const int idx = (int)c->sp.size();
    int cnt[2] = {(int)n, 0};
    HIPCHK(c, hipMemcpyAsync(&small_of(c)->count[idx], &cnt[0], sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(&small_of(c)->sorted[idx], &cnt[1], sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pused += bufs->capacity;
    c->sp.push_back(s);
    if (species_out) *species_out = idx;
    return PIC_OK;
}

pic_status pic_gather_push(pic_ctx* c, int32_t s) {
    PICCHK(check_species(c, s));
    Species& sp = c->sp[s];
    HIPCHK(c, launch_gather_push(c->g, fields_of(c), dev_of(c, sp), prev_of(c, sp), &small_of(c)->count[s],
                                 (int)sp.bound, &small_of(c)->err, c->stream));
    sp.prev_valid = true;
    c->mid_step = true;
    return PIC_OK;
}

pic_status pic_deposit(pic_ctx* c, int32_t s) {
    PICCHK(check_species(c, s));
    Species& sp = c->sp[s];
    if (!sp.prev_valid) return fail(c, PIC_ESTATE, "deposit needs a preceding gather_push");
    HIPCHK(c, launch_deposit(c->g, dev_of(c, sp), prev_of(c, sp), &small_of(c)->count[s], (int)sp.bound, acc_of(c),
                             c->stream));
    double sc[3];
    jscale(c, sc);
    HIPCHK(c, launch_jfinal(c->g, acc_of(c), c->f.J, sc, 0, c->stream));
    c->j_filtered = false;
    return PIC_OK;
}

pic_status pic_field_step(pic_ctx* c) {
    if (!c) return PIC_EINVAL;
    float* Juse[3] = {c->f.J[0], c->f.J[1], c->f.J[2]};
    PICCHK(filter_in_place(c));
    PICCHK(field_update(c, Juse));
    HIPCHK(c, launch_zero_u64(acc_of(c), 3 * (int64_t)c->g.ncell, c->stream));
    c->mid_step = false;
    return end_step(c);
}

pic_status pic_step(pic_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return PIC_EINVAL;
    for (int32_t it = 0; it < nsteps; ++it) {
        for (int32_t s = 0; s < (int32_t)c->sp.size(); ++s) {
            Species& sp = c->sp[s];
            if (sp.bound == 0) {            // no particle can exist: nothing to sort, push or deposit
                sp.prev_valid = false;
                continue;
            }
            hipEvent_t t0, t1, t2;
            bool gather = false;
            if (!sp.sorted || c->step - sp.sort_step >= c->tl.sort_interval) {
                PICCHK(prof_mark(c, &t0));
                PICCHK(sort_species(c, s, false));
                PICCHK(prof_end(c, PH_SORT, t0));
                if (c->prof.on) c->prof.sorts += 1;
                gather = true;
            }
            Small* sm = small_of(c);
            PICCHK(prof_mark(c, &t1));
            int* rest_idx = reinterpret_cast<int*>(c->ws + c->L.sort_rank) + sp.base;
            const SpeciesDev pre = dev_from(c, sp, sp.alt);   // the pre-sort set after a sort
            HIPCHK(c, launch_pic_tile(c->g, c->tl.t, c->tl.guard, c->tl.threads, fields_of(c), dev_of(c, sp),
                                      gather ? &pre : nullptr, toff_of(c, s), acc_of(c), &sm->err, &sm->rest_n[s],
                                      rest_idx, c->stream));
            PICCHK(prof_end(c, PH_TILE, t1));
            if (c->prof.on) c->prof.tiles += 1;
            PICCHK(prof_mark(c, &t2));
            HIPCHK(c, launch_tile_rest(c->g, fields_of(c), dev_of(c, sp), &sm->sorted[s], &sm->count[s],
                                       &sm->rest_n[s], rest_idx, acc_of(c), &sm->err, c->stream));
            PICCHK(prof_end(c, PH_LOOSE, t2));
            sp.prev_valid = false;
        }
        PICCHK(finish_step(c));
    }
    return PIC_OK;
}

pic_status pic_sort(pic_ctx* c, int32_t s) {
    PICCHK(check_species(c, s));
    return sort_species(c, s, true);
}

pic_status pic_species_view(pic_ctx* c, int32_t s, pic_species_bufs* out, int64_t* n_live) {
    PICCHK(check_species(c, s));
    int cnt = 0;
    HIPCHK(c, hipMemcpyAsync(&cnt, &small_of(c)->count[s], sizeof(int), hipMemcpyDeviceToHost, c->stream));
    pic_status st = device_errors(c);
    if (out) *out = c->sp[s].cur;
    if (n_live) *n_live = cnt;
    return st;
}

pic_status pic_continuity(pic_ctx* c, int32_t s, double* resid, double* max_abs_j) {
    PICCHK(check_species(c, s));
    Species& sp = c->sp[s];
    if (!sp.prev_valid) return fail(c, PIC_ESTATE, "continuity needs a preceding gather_push and deposit");
    double* rho = reinterpret_cast<double*>(c->ws + c->L.rho);
    Small* sm = small_of(c);
    HIPCHK(c, hipMemsetAsync(rho, 0, (size_t)c->g.ncell * 8, c->stream));
    HIPCHK(c, hipMemsetAsync(&sm->contmax, 0, 8, c->stream));
    HIPCHK(c, hipMemsetAsync(&sm->jmax, 0, 4, c->stream));
    HIPCHK(c, hipMemsetAsync(sm->red, 0, sizeof sm->red, c->stream));
    SpeciesDev d = dev_of(c, sp);
    PrevDev pv = prev_of(c, sp);
    HIPCHK(c, launch_rho(c->g, d.cell, d.off, d.w, sp.user.q, 1.0, &sm->count[s], (int)sp.bound, rho, c->stream));
    HIPCHK(c, launch_rho(c->g, pv.cell, pv.off, d.w, sp.user.q, -1.0, &sm->count[s], (int)sp.bound, rho, c->stream));
    HIPCHK(c, launch_continuity(c->g, rho, c->f.J, c->desc.d[0] / c->desc.dt, c->desc.d[0] / c->desc.d[1],
                                c->desc.d[0] / c->desc.d[2], c->j_filtered, &sm->contmax,
                                c->stream));
    FieldPtrs f = fields_of(c);
    HIPCHK(c, launch_diag_fields(c->g, f.E, f.B, c->f.J, 1.0, sm->red, &sm->jmax, c->stream));
    unsigned long long cm = 0;
    unsigned int jm = 0;
    HIPCHK(c, hipMemcpyAsync(&cm, &sm->contmax, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&jm, &sm->jmax, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double r;
    memcpy(&r, &cm, 8);
    float j;
    memcpy(&j, &jm, 4);
    if (resid) *resid = r;
    if (max_abs_j) *max_abs_j = j;
    return device_errors(c);
}

pic_status pic_continuity_noalloc(pic_ctx* c, int32_t s, double* resid, double* max_abs_j) {
    PICCHK(check_species(c, s));
    if (c->g.ncell > kNoAllocMaxCells)
        return fail(c, PIC_EINVAL, "grid of %d cells exceeds the %d cells of the allocation-free continuity check",
                    c->g.ncell, kNoAllocMaxCells);
    Species& sp = c->sp[s];
    if (!sp.prev_valid) return fail(c, PIC_ESTATE, "continuity needs a preceding gather_push and deposit");
    void* base = nullptr;
    HIPCHK(c, noalloc_scratch(&base));
    NoAllocHead* head = reinterpret_cast<NoAllocHead*>(base);
    double* rho = reinterpret_cast<double*>(reinterpret_cast<char*>(base) + kNoAllocRhoOffset);
    // clear the head and this grid's density with a fill kernel (no memset node)
    HIPCHK(c, launch_zero_u64(reinterpret_cast<unsigned long long*>(base),
                              (int64_t)(kNoAllocRhoOffset / 8) + c->g.ncell, c->stream));
    SpeciesDev d = dev_of(c, sp);
    PrevDev pv = prev_of(c, sp);
    Small* sm = small_of(c);
    HIPCHK(c, launch_rho(c->g, d.cell, d.off, d.w, sp.user.q, 1.0, &sm->count[s], (int)sp.bound, rho, c->stream));
    HIPCHK(c, launch_rho(c->g, pv.cell, pv.off, d.w, sp.user.q, -1.0, &sm->count[s], (int)sp.bound, rho, c->stream));
    HIPCHK(c, launch_continuity(c->g, rho, c->f.J, c->desc.d[0] / c->desc.dt, c->desc.d[0] / c->desc.d[1],
                                c->desc.d[0] / c->desc.d[2], c->j_filtered, &head->contmax,
                                c->stream));
    FieldPtrs f = fields_of(c);
    HIPCHK(c, launch_diag_fields(c->g, f.E, f.B, c->f.J, 1.0, head->red, &head->jmax, c->stream));
    unsigned long long cm = 0;
    unsigned int jm = 0;
    HIPCHK(c, hipMemcpyAsync(&cm, &head->contmax, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&jm, &head->jmax, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double r;
    memcpy(&r, &cm, 8);
    float j;
    memcpy(&j, &jm, 4);
    if (resid) *resid = r;
    if (max_abs_j) *max_abs_j = j;
    return device_errors(c);
}

pic_status pic_reduce(pic_ctx* c, pic_diag* out) {
    if (!c || !out) return PIC_EINVAL;
    Small* sm = small_of(c);
    HIPCHK(c, hipMemsetAsync(sm->red, 0, sizeof sm->red, c->stream));
    HIPCHK(c, hipMemsetAsync(&sm->live, 0, 8, c->stream));
    HIPCHK(c, hipMemsetAsync(&sm->jmax, 0, 4, c->stream));
    const double dv = c->desc.d[0] * c->desc.d[1] * c->desc.d[2];
    for (int32_t s = 0; s < (int32_t)c->sp.size(); ++s) {
        Species& sp = c->sp[s];
        HIPCHK(c, launch_diag_particles(c->g, dev_of(c, sp), sp.user.q, sp.user.m, dv, &sm->count[s], (int)sp.bound,
                                        sm->red, &sm->live, c->stream));
    }
    FieldPtrs f = fields_of(c);
    HIPCHK(c, launch_diag_fields(c->g, f.E, f.B, c->f.J, dv, sm->red, &sm->jmax, c->stream));
    double red[4];
    unsigned long long live = 0;
    unsigned int jm = 0;
    HIPCHK(c, hipMemcpyAsync(red, sm->red, sizeof red, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&live, &sm->live, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&jm, &sm->jmax, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float j;
    memcpy(&j, &jm, 4);
    out->charge = red[0];
    out->e_kin = red[1];
    out->e_field = red[2];
    out->max_abs_J = j;
    out->n_particles = (int64_t)live;
    out->step = c->step;
    return device_errors(c);
}

pic_status pic_sync(pic_ctx* c) {
    if (!c) return PIC_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return device_errors(c);
}

pic_status pic_set_laser(pic_ctx* c, const pic_laser_desc* L) {
    if (!c) return PIC_EINVAL;
    if (!L) {
        c->has_laser = false;
        return PIC_OK;
    }
    if (L->src_x < 1 || L->src_x >= c->g.n[0] - 1) return fail(c, PIC_EINVAL, "laser source plane outside [1, nx-1)");
    if (!(L->fwhm > 0.0) || !(L->waist > 0.0) || !isfinite(L->a0) || !isfinite(L->omega0) || !isfinite(L->t_peak) ||
        !isfinite(L->t_end))
        return fail(c, PIC_EINVAL, "invalid laser parameters");
    if (c->g.window && c->window_start != INT64_MAX && L->t_end > c->window_start * c->desc.dt)
        return fail(c, PIC_EINVAL, "the window would move while the laser source is active");
    c->laser = *L;
    c->has_laser = true;
    return PIC_OK;
}

pic_status pic_set_plasma(pic_ctx* c, int32_t s, const pic_plasma_desc* P) {
    PICCHK(check_species(c, s));
    if (!P) {
        c->has_plasma[s] = false;
        return PIC_OK;
    }
    for (int a = 0; a < 3; ++a)
        if (P->ppc[a] < 1 || P->ppc[a] > 16) return fail(c, PIC_EINVAL, "lattice particles per cell outside 1..16");
    if (!(P->ramp >= 0.0) || !isfinite(P->x_start) || !(P->n_plateau >= 0.0) || !isfinite(P->n_plateau))
        return fail(c, PIC_EINVAL, "invalid plasma profile");
    PlasmaDev& d = c->plasma[s];
    d.x_start = P->x_start;
    d.ramp = P->ramp;
    d.n_plateau = P->n_plateau;
    for (int a = 0; a < 3; ++a) d.ppc[a] = P->ppc[a];
    c->has_plasma[s] = true;
    return PIC_OK;
}

pic_status pic_inject_plasma(pic_ctx* c, int32_t s, int32_t xb, int32_t xe) {
    PICCHK(check_species(c, s));
    if (!c->has_plasma[s]) return fail(c, PIC_ESTATE, "species %d has no plasma profile", s);
    if (xb < 0 || xe > c->g.n[0] || xb > xe) return fail(c, PIC_EINVAL, "slab outside the grid");
    return inject_slab(c, s, xb, xe);
}

pic_status pic_set_window(pic_ctx* c, int64_t start_step) {
    if (!c) return PIC_EINVAL;
    if (!c->g.window) return fail(c, PIC_ESTATE, "the grid has no moving window (bc_x)");
    if (fabs(c->desc.dt - c->desc.d[0]) > 1e-12 * c->desc.d[0])
        return fail(c, PIC_EINVAL, "a window moving one cell per step at c needs c dt = dx");
    if (start_step < 0) return fail(c, PIC_EINVAL, "negative start step");
    if (c->has_laser && c->laser.t_end > start_step * c->desc.dt)
        return fail(c, PIC_EINVAL, "the window would move while the laser source is active");
    c->window_start = start_step;
    return PIC_OK;
}

pic_status pic_window_state(pic_ctx* c, int64_t* shift, int32_t* origin) {
    if (!c) return PIC_EINVAL;
    if (shift) *shift = c->shift;
    if (origin) *origin = c->g.origin;
    return PIC_OK;
}

size_t pic_pml_bytes(const pic_grid_desc* desc, const pic_pml_desc* pml) {
    PmlLayout L;
    return pml_layout(desc, pml, &L) ? L.total : 0;
}

pic_status pic_set_pml(pic_ctx* c, const pic_pml_desc* p, void* buffer, size_t bytes) {
    if (!c || !p) return PIC_EINVAL;
    if (c->mid_step) return fail(c, PIC_ESTATE, "absorbing layer changed inside a split-path step");
    if (p->layers == 0) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->g.pml = 0;
        c->pml = PmlDev{};
        c->pml_buf = nullptr;
        c->pml_state_bytes = 0;
        return PIC_OK;
    }
    PmlLayout L;
    if (!pml_layout(&c->desc, p, &L))
        return fail(c, PIC_EINVAL, "absorbing layer of %d cells: need 8 <= layers and 2 layers + 1 <= n[1], n[2]",
                    p->layers);
    if (!buffer || (reinterpret_cast<uintptr_t>(buffer) & (kAlign - 1)) != 0)
        return fail(c, PIC_EINVAL, "absorbing layer buffer null or not 256-byte aligned");
    if (bytes < L.total) return fail(c, PIC_ENOMEM, "absorbing layer needs %zu bytes, buffer has %zu", L.total, bytes);
    const double grade = p->grade > 0.0 ? p->grade : 3.0;
    double smax[2];
    for (int a = 0; a < 2; ++a) {
        smax[a] = p->sigma_max[a] > 0.0 ? p->sigma_max[a] : 0.8 * (grade + 1.0) / c->desc.d[1 + a];
        if (!isfinite(smax[a]) || !isfinite(grade) || grade > 16.0)
            return fail(c, PIC_EINVAL, "invalid absorbing layer conductivity or grade");
    }
    // coefficient table: [axis][kind][b, b - 1][2L] (see PmlDev)
    const int Ly = p->layers, L2 = 2 * Ly;
    std::vector<float> coef((size_t)16 * Ly);
    for (int axis = 0; axis < 2; ++axis) {
        const int n = c->desc.n[1 + axis];
        for (int kind = 0; kind < 2; ++kind)
            for (int l = 0; l < L2; ++l) {
                const int j = l < Ly ? l : n - L2 + l;
                const double pos = kind == 0 ? j + 0.5 : (double)j;
                const double sdt = pml_sigma_at(smax[axis], grade, Ly, n, pos) * c->desc.dt;
                coef[(size_t)((axis * 2 + kind) * 2 + 0) * L2 + l] = (float)exp(-sdt);
                coef[(size_t)((axis * 2 + kind) * 2 + 1) * L2 + l] = (float)expm1(-sdt);
            }
    }
    char* base = reinterpret_cast<char*>(buffer);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemsetAsync(base, 0, L.total, c->stream));
    HIPCHK(c, hipMemcpyAsync(base + L.coef, coef.data(), coef.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pml_desc = *p;
    c->pml.coef = reinterpret_cast<const float*>(base + L.coef);
    for (int a = 0; a < 4; ++a) {
        c->pml.y[a] = reinterpret_cast<float*>(base + L.y[a]);
        c->pml.z[a] = reinterpret_cast<float*>(base + L.z[a]);
    }
    c->pml.L = Ly;
    c->pml_buf = base;
    c->pml_state_bytes = L.total - L.y[0];
    c->g.pml = Ly;
    // species are re-sorted at their next step (the sort drops the layer's particles)
    for (auto& sp : c->sp) sp.sorted = false;
    return PIC_OK;
}

pic_status pic_checkpoint_bytes(pic_ctx* c, size_t* bytes) {
    if (!c || !bytes) return PIC_EINVAL;
    int64_t count[kMaxSpecies] = {};
    PICCHK(exact_counts(c, count));
    *bytes = ckpt_bytes(c, count);
    return PIC_OK;
}

pic_status pic_copy_out(pic_ctx* c, void* host_blob, size_t bytes) {
    if (!c || !host_blob) return PIC_EINVAL;
    if (c->mid_step) return fail(c, PIC_ESTATE, "checkpoint inside a split-path step (gather_push without field_step)");
    int64_t count[kMaxSpecies] = {};
    PICCHK(exact_counts(c, count));
    const size_t need = ckpt_bytes(c, count);
    if (bytes < need) return fail(c, PIC_ENOMEM, "checkpoint needs %zu bytes, blob has %zu", need, bytes);
    CkptHeader h;
    memset(&h, 0, sizeof h);
    h.magic = kCkptMagic;
    h.version = kCkptVersion;
    h.nspecies = (uint32_t)c->sp.size();
    for (int a = 0; a < 3; ++a) {
        h.n[a] = c->desc.n[a];
        h.d[a] = c->desc.d[a];
    }
    h.origin = c->g.origin;
    h.solver = c->desc.solver;
    h.bc_x = c->desc.bc_x;
    h.pml_layers = c->g.pml;
    h.dt = c->desc.dt;
    h.step = c->step;
    h.shift = c->shift;
    for (size_t s = 0; s < c->sp.size(); ++s) h.count[s] = count[s];
    char* p = reinterpret_cast<char*>(host_blob);
    memcpy(p, &h, sizeof h);
    p += sizeof h;
    const size_t fbytes = (size_t)c->g.ncell * 4;
    float* const* F[3] = {c->f.E, c->f.B, c->f.J};
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
            HIPCHK(c, hipMemcpyAsync(p, F[k][a], fbytes, hipMemcpyDeviceToHost, c->stream));
            p += fbytes;
        }
    if (c->g.pml) {
        HIPCHK(c, hipMemcpyAsync(p, c->pml.y[0], c->pml_state_bytes, hipMemcpyDeviceToHost, c->stream));
        p += c->pml_state_bytes;
    }
    for (size_t s = 0; s < c->sp.size(); ++s) {
        void* arr[kCkptArrays];
        ckpt_arrays(c->sp[s].cur, arr);
        const size_t pb = (size_t)count[s] * 4;
        for (int k = 0; k < kCkptArrays; ++k) {
            if (pb) HIPCHK(c, hipMemcpyAsync(p, arr[k], pb, hipMemcpyDeviceToHost, c->stream));
            p += pb;
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

pic_status pic_copy_in(pic_ctx* c, const void* host_blob, size_t bytes) {
    if (!c || !host_blob) return PIC_EINVAL;
    if (bytes < sizeof(CkptHeader)) return fail(c, PIC_EINVAL, "checkpoint blob shorter than its header");
    CkptHeader h;
    memcpy(&h, host_blob, sizeof h);
    if (h.magic != kCkptMagic || h.version != kCkptVersion) return fail(c, PIC_EINVAL, "not a checkpoint of this library");
    for (int a = 0; a < 3; ++a)
        if (h.n[a] != c->desc.n[a] || h.d[a] != c->desc.d[a])
            return fail(c, PIC_EINVAL, "checkpoint grid differs from the context's");
    if (h.dt != c->desc.dt || h.solver != c->desc.solver || h.bc_x != c->desc.bc_x)
        return fail(c, PIC_EINVAL, "checkpoint time step, solver or x boundary differs from the context's");
    if (h.pml_layers != c->g.pml)
        return fail(c, PIC_EINVAL, "checkpoint absorbing layer (%d cells) differs from the context's (%d)", h.pml_layers,
                    c->g.pml);
    if (h.nspecies != c->sp.size()) return fail(c, PIC_EINVAL, "checkpoint has %u species, context %zu", h.nspecies,
                                                c->sp.size());
    if (h.origin < 0 || h.origin >= c->g.n[0] || h.step < 0 || h.shift < 0 || (!c->g.window && (h.shift || h.origin)))
        return fail(c, PIC_EINVAL, "invalid step or window state in the checkpoint");
    for (size_t s = 0; s < c->sp.size(); ++s)
        if (h.count[s] < 0 || h.count[s] > c->sp[s].user.capacity)
            return fail(c, PIC_ENOMEM, "species %zu: %lld particles exceed capacity %lld", s, (long long)h.count[s],
                        (long long)c->sp[s].user.capacity);
    if (bytes < ckpt_bytes(c, h.count)) return fail(c, PIC_EINVAL, "checkpoint blob truncated");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const char* p = reinterpret_cast<const char*>(host_blob) + sizeof h;
    const size_t fbytes = (size_t)c->g.ncell * 4;
    float* const* F[3] = {c->f.E, c->f.B, c->f.J};
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
            HIPCHK(c, hipMemcpyAsync(F[k][a], p, fbytes, hipMemcpyHostToDevice, c->stream));
            p += fbytes;
        }
    if (c->g.pml) {
        HIPCHK(c, hipMemcpyAsync(c->pml.y[0], p, c->pml_state_bytes, hipMemcpyHostToDevice, c->stream));
        p += c->pml_state_bytes;
    }
    Small* sm = small_of(c);
    for (size_t s = 0; s < c->sp.size(); ++s) {
        Species& sp = c->sp[s];
        // the caller's arrays hold the data again; the workspace set is the spare
        if (sp.cur.cell != sp.user.cell) std::swap(sp.cur, sp.alt);
        void* arr[kCkptArrays];
        ckpt_arrays(sp.cur, arr);
        const size_t pb = (size_t)h.count[s] * 4;
        for (int k = 0; k < kCkptArrays; ++k) {
            if (pb) HIPCHK(c, hipMemcpyAsync(arr[k], p, pb, hipMemcpyHostToDevice, c->stream));
            p += pb;
        }
        int cnt[2] = {(int)h.count[s], 0};
        HIPCHK(c, hipMemcpyAsync(&sm->count[s], &cnt[0], sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(&sm->sorted[s], &cnt[1], sizeof(int), hipMemcpyHostToDevice, c->stream));
        sp.bound = h.count[s];
        sp.sorted = false;
        sp.prev_valid = false;
    }
    HIPCHK(c, launch_zero_u64(acc_of(c), 3 * (int64_t)c->g.ncell, c->stream));
    c->step = h.step;
    c->shift = h.shift;
    c->g.origin = h.origin;
    c->mid_step = false;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

// ---- run diagnostics ---------------------------------------------------------


pic_status pic_axis_line(pic_ctx* c, int32_t comp, double yc, double zc, double* host_line) {
    if (!c || !host_line) return PIC_EINVAL;
    if (comp < 0 || comp > 5) return fail(c, PIC_EINVAL, "field component %d outside 0..5", comp);
    if (!isfinite(yc) || !isfinite(zc)) return fail(c, PIC_EINVAL, "non-finite axis position");
    int j0, k0;
    double ty, tz;
    axis_weights(c, comp, yc, zc, &j0, &k0, &ty, &tz);
    double* line = diag_words(c) + kDiagWords;
    HIPCHK(c, launch_axis_line(c->g, field_comp(c, comp), j0, k0, ty, tz, line, c->stream));
    HIPCHK(c, hipMemcpyAsync(host_line, line, (size_t)c->g.n[0] * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

pic_status pic_accelerating_length(pic_ctx* c, double yc, double zc, double x_from, double* length) {
    if (!c || !length) return PIC_EINVAL;
    const int nx = c->g.n[0];
    std::vector<double> line((size_t)nx);
    PICCHK(pic_axis_line(c, 0, yc, zc, line.data()));
    // E_x samples sit at (i + 1/2) dx in window coordinates
    const double dx = c->desc.d[0];
    auto xs = [&](int i) { return (i + 0.5) * dx; };
    int i = (int)floor(x_from / dx - 0.5);
    if (i >= nx) i = nx - 1;
    *length = 0.0;
    if (i < 0) return PIC_OK;
    const int start = i;
    while (i >= 0 && line[i] >= 0.0) --i;
    if (i < 0) return PIC_OK;
    const int hi = i;
    while (i >= 0 && line[i] < 0.0) --i;
    const int lo = i + 1;
    auto crossing = [&](int a, int b) { return xs(a) + (xs(b) - xs(a)) * line[a] / (line[a] - line[b]); };
    double front;
    if (hi < start)
        front = crossing(hi + 1, hi);
    else
        front = (hi + 1 >= nx || line[hi + 1] < 0.0) ? x_from : crossing(hi + 1, hi);
    const double rear = lo >= 1 ? crossing(lo - 1, lo) : xs(lo);
    *length = front - rear;
    return PIC_OK;
}

pic_status pic_spectrum(pic_ctx* c, int32_t s, int32_t quantity, double lo, double hi, int32_t nbins,
                        double* host_charge, int64_t* host_count) {
    PICCHK(check_species(c, s));
    if (!host_charge) return PIC_EINVAL;
    if (quantity != 0 && quantity != 1) return fail(c, PIC_EINVAL, "spectrum quantity must be 0 (gamma-1) or 1 (u_x)");
    if (nbins < 1 || nbins > kDiagBins) return fail(c, PIC_EINVAL, "spectrum bins outside 1..%d", kDiagBins);
    if (!(hi > lo) || !isfinite(lo) || !isfinite(hi)) return fail(c, PIC_EINVAL, "spectrum range must have hi > lo");
    double* charge = reinterpret_cast<double*>(c->ws + c->L.diag);
    unsigned long long* count = reinterpret_cast<unsigned long long*>(charge + kDiagBins);
    HIPCHK(c, launch_zero_u64(reinterpret_cast<unsigned long long*>(charge), 2 * kDiagBins, c->stream));
    Species& sp = c->sp[s];
    const double dv = c->desc.d[0] * c->desc.d[1] * c->desc.d[2];
    HIPCHK(c, launch_spectrum(c->g, dev_of(c, sp), &small_of(c)->count[s], (int)sp.bound, quantity, lo, hi, nbins,
                              fabs(sp.user.q) * dv, charge, count, c->stream));
    HIPCHK(c, hipMemcpyAsync(host_charge, charge, (size_t)nbins * 8, hipMemcpyDeviceToHost, c->stream));
    if (host_count) HIPCHK(c, hipMemcpyAsync(host_count, count, (size_t)nbins * 8, hipMemcpyDeviceToHost, c->stream));
    return device_errors(c);
}

pic_status pic_beam_moments(pic_ctx* c, int32_t s, double ux_min, pic_beam_diag* out) {
    PICCHK(check_species(c, s));
    if (!out) return PIC_EINVAL;
    double* sums = diag_words(c);
    HIPCHK(c, launch_zero_u64(reinterpret_cast<unsigned long long*>(sums), 13, c->stream));
    Species& sp = c->sp[s];
    HIPCHK(c, launch_beam_moments(c->g, dev_of(c, sp), &small_of(c)->count[s], (int)sp.bound, ux_min, c->desc.d[1],
                                  c->desc.d[2], sums, c->stream));
    double h[13];
    HIPCHK(c, hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, c->stream));
    PICCHK(device_errors(c));
    const double dv = c->desc.d[0] * c->desc.d[1] * c->desc.d[2];
    memset(out, 0, sizeof *out);
    out->count = (int64_t)h[12];
    out->charge = fabs(sp.user.q) * dv * h[0];
    if (h[0] > 0.0) {
        const double W = h[0];
        out->mean_ux = h[1] / W;
        double eps[2];
        for (int a = 0; a < 2; ++a) {
            const double* m = h + 2 + 5 * a;
            const double mr = m[0] / W, mr2 = m[1] / W, mp = m[2] / W, mp2 = m[3] / W, mpr = m[4] / W;
            const double var_p = mp2 - mp * mp, var_r = mr2 - mr * mr, cov = mpr - mr * mp;
            const double v = var_p * var_r - cov * cov;
            eps[a] = v > 0.0 ? sqrt(v) : 0.0;
            out->mean_r[a] = mr;
            out->rms_r[a] = var_r > 0.0 ? sqrt(var_r) : 0.0;
            out->rms_p[a] = var_p > 0.0 ? sqrt(var_p) : 0.0;
        }
        out->eps_ny = eps[0];
        out->eps_nz = eps[1];
    }
    return PIC_OK;
}

pic_status pic_select_particles(pic_ctx* c, int32_t s, double ux_min, int64_t cap, int32_t* host_id, double* host_x,
                                float* host_ux, int64_t* n_selected) {
    PICCHK(check_species(c, s));
    if (cap < 0 || (cap > 0 && (!host_id || !host_x || !host_ux))) return PIC_EINVAL;
    Species& sp = c->sp[s];
    int* counter = reinterpret_cast<int*>(diag_words(c) + 16);
    HIPCHK(c, launch_zero_u64(reinterpret_cast<unsigned long long*>(counter), 1, c->stream));
    // staging: the species' spare particle arrays (free between steps)
    const pic_species_bufs& o = sp.alt;
    HIPCHK(c, launch_select(c->g, dev_of(c, sp), &small_of(c)->count[s], (int)sp.bound, ux_min, o.cell, o.off[0],
                            o.u[0], o.id, counter, c->stream));
    int nsel = 0;
    HIPCHK(c, hipMemcpyAsync(&nsel, counter, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    PICCHK(device_errors(c));
    if (n_selected) *n_selected = nsel;
    const int64_t k = nsel < cap ? nsel : cap;
    if (k > 0) {
        std::vector<int32_t> cell((size_t)k);
        std::vector<float> off((size_t)k);
        HIPCHK(c, hipMemcpyAsync(cell.data(), o.cell, (size_t)k * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(off.data(), o.off[0], (size_t)k * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(host_ux, o.u[0], (size_t)k * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(host_id, o.id, (size_t)k * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int nx = c->g.n[0];
        for (int64_t q = 0; q < k; ++q) {
            int xw = cell[q] % nx;
            if (c->g.window) xw = (xw - c->g.origin + nx) % nx;
            host_x[q] = ((double)xw + (double)off[q]) * c->desc.d[0];
        }
    }
    return PIC_OK;
}

pic_status pic_field_moments(pic_ctx* c, int32_t transverse_only, double* host_out) {
    if (!c || !host_out) return PIC_EINVAL;
    double* sums = diag_words(c) + 24;
    HIPCHK(c, launch_zero_u64(reinterpret_cast<unsigned long long*>(sums), 3, c->stream));
    const int mask = transverse_only ? 0x36 : 0x3f;   // E_y, E_z, B_y, B_z or all six
    FieldPtrs f = fields_of(c);
    HIPCHK(c, launch_field_moments(c->g, f.E, f.B, mask, c->desc.d[0], c->desc.d[0] * c->desc.d[1] * c->desc.d[2],
                                   sums, c->stream));
    HIPCHK(c, hipMemcpyAsync(host_out, sums, 3 * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

pic_status pic_set_tiling(pic_ctx* c, const pic_tiling* t) {
    if (!c || !t) return PIC_EINVAL;
    const char* why = validate_tiling(c->desc.n, t->tile, t->guard, t->threads, t->interleave, t->sort_interval);
    if (why) return fail(c, PIC_EINVAL, "%s", why);
    for (int a = 0; a < 3; ++a) c->desc.tile[a] = t->tile[a];
    c->desc.guard = t->guard;
    c->desc.threads = t->threads;
    c->desc.interleave = t->interleave;
    c->desc.sort_interval = t->sort_interval;
    c->tl = tiling_of(&c->desc);
    for (auto& sp : c->sp) sp.sorted = false;
    return PIC_OK;
}

pic_status pic_profile_enable(pic_ctx* c, int32_t enable) {
    if (!c) return PIC_EINVAL;
    HIPCHK(c, c->prof.enable(c->stream, enable != 0));
    return PIC_OK;
}

pic_status pic_profile_read(pic_ctx* c, pic_profile* out) {
    if (!c || !out) return PIC_EINVAL;
    HIPCHK(c, c->prof.read(c->stream, out));
    return PIC_OK;
}

pic_status pic_denoiser_set(pic_ctx* c, const float* weights, const float* biases, const float* scale) {
    if (!c || !weights || !biases || !scale) return PIC_EINVAL;
    if (c->desc.jpost != PIC_JPOST_DENOISER)
        return fail(c, PIC_ESTATE, "the grid was not created with the denoiser current post-processing");
    for (int d = 0; d < 3; ++d)
        if (!(scale[d] > 0.0f) || !isfinite(scale[d])) return fail(c, PIC_EINVAL, "scales must be positive and finite");
    const size_t nw1 = 32 * 3 * 27, nw2 = 32 * 32 * 27, nw3 = 3 * 32 * 27;
    for (size_t i = 0; i < nw1 + nw2 + nw3; ++i)
        if (!isfinite(weights[i])) return fail(c, PIC_EINVAL, "non-finite weight");
    for (size_t i = 0; i < 67; ++i)
        if (!isfinite(biases[i])) return fail(c, PIC_EINVAL, "non-finite bias");
    // pack: bf16 round to nearest even
    auto bf = [](float v) -> uint16_t {
        uint32_t u;
        memcpy(&u, &v, 4);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    };
    std::vector<uint16_t> w((kDnW1 + kDnW2 + kDnW3), 0);
    uint16_t* w1 = w.data();
    uint16_t* w2 = w1 + kDnW1;
    uint16_t* w3 = w2 + kDnW2;
    const float* W1 = weights;
    const float* W2 = W1 + nw1;
    const float* W3 = W2 + nw2;
    for (int co = 0; co < 32; ++co)
        for (int ci = 0; ci < 3; ++ci)
            for (int t = 0; t < 27; ++t) w1[co * 128 + t * 4 + ci] = bf(W1[(co * 3 + ci) * 27 + t]);
    for (int t = 0; t < 27; ++t)
        for (int co = 0; co < 32; ++co)
            for (int ci = 0; ci < 32; ++ci) w2[(t * 32 + co) * 32 + ci] = bf(W2[(co * 32 + ci) * 27 + t]);
    // W3 for the folded last layer: fragment (tap column zx, halo row r), column
    // 4 blk + co carries tap (dz, r - blk, dx) when 0 <= r - blk <= 2
    for (int zx = 0; zx < 9; ++zx)
        for (int r = 0; r < 6; ++r)
            for (int blk = 0; blk < 4; ++blk) {
                const int dy = r - blk;
                if (dy < 0 || dy > 2) continue;
                const int t = (zx / 3) * 9 + dy * 3 + zx % 3;
                for (int co = 0; co < 3; ++co)
                    for (int ci = 0; ci < 32; ++ci)
                        w3[((zx * 6 + r) * 16 + blk * 4 + co) * 32 + ci] = bf(W3[(co * 32 + ci) * 27 + t]);
            }
    std::vector<float> b(kDnBias, 0.0f);
    for (int i = 0; i < 32; ++i) b[i] = biases[i];
    for (int i = 0; i < 32; ++i) b[32 + i] = biases[32 + i];
    for (int i = 0; i < 3; ++i) b[64 + i] = biases[64 + i];
    char* dst = c->ws + c->L.dn_w;
    const size_t wbytes = w.size() * 2;
    HIPCHK(c, hipMemcpyAsync(dst, w.data(), wbytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dst + wbytes, b.data(), kDnBias * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    DenoiseWeights& d = c->dn;
    d.w1 = reinterpret_cast<const __bf16*>(dst);
    d.w2 = d.w1 + kDnW1;
    d.w3 = d.w2 + kDnW2;
    d.b1 = reinterpret_cast<const float*>(dst + wbytes);
    d.b2 = d.b1 + 32;
    d.b3 = d.b2 + 32;
    for (int i = 0; i < 3; ++i) {
        d.scale[i] = scale[i];
        d.inv_d[i] = (float)(1.0 / c->desc.d[i]);
    }
    d.sigma = (float)(c->desc.d[0] * ((double)scale[0] + scale[1] + scale[2]) / 3.0);
    c->has_dn = true;
    return PIC_OK;
}

pic_status pic_current_filter(pic_ctx* c) {
    if (!c) return PIC_EINVAL;
    return filter_in_place(c);
}

const char* pic_last_error(const pic_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

void pic_destroy(pic_ctx* c) { delete c; }

size_t pic_batch_workspace_bytes(int32_t n) {
    if (n < 1) return 0;
    return (size_t)kBatchSlots * batch_slot_bytes(n);
}

pic_status pic_batch_create(pic_batch** out, pic_ctx* const* members, int32_t n, void* workspace,
                            size_t workspace_bytes, void* stream) {
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    if (!members || n < 1 || !workspace) return PIC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0) return PIC_EINVAL;
    if (workspace_bytes < pic_batch_workspace_bytes(n)) return PIC_ENOMEM;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int32_t i = 0; i < n; ++i) {
        if (!members[i]) return PIC_EINVAL;
        if (members[i]->stream != st) return PIC_EINVAL;
        if (members[i]->sp.empty() || members[i]->sp.size() != members[0]->sp.size()) return PIC_EINVAL;
        if (members[i]->g.pml) return PIC_EINVAL;   // the batched field kernels have no absorbing layer
        for (int32_t k = 0; k < i; ++k)
            if (members[k] == members[i]) return PIC_EINVAL;
    }
    pic_batch* b = new (std::nothrow) pic_batch();
    if (!b) return PIC_ENOMEM;
    b->m.assign(members, members + n);
    b->nsp = (int)members[0]->sp.size();
    b->stream = st;
    b->ws = reinterpret_cast<char*>(workspace);
    b->tab_bytes = batch_tab_bytes(n);
    b->slot_bytes = batch_slot_bytes(n);
    hipError_t e = hipHostMalloc((void**)&b->host, (size_t)kBatchSlots * b->slot_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        b->host = nullptr;
        delete b;
        return PIC_EDEVICE;
    }
    b->ev.assign(kBatchSlots, nullptr);
    b->used.assign(kBatchSlots, false);
    for (int k = 0; k < kBatchSlots && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete b;
        return PIC_EDEVICE;
    }
    *out = b;
    return PIC_OK;
}

pic_status pic_batch_step(pic_batch* b, int32_t nsteps) {
    if (!b || nsteps < 0) return PIC_EINVAL;
    for (pic_ctx* c : b->m) {
        if (c->desc.jpost == PIC_JPOST_DENOISER)
            return bfail(b, PIC_EINVAL, "the batch runs the plain and binomial current paths only");
        if (c->g.pml) return bfail(b, PIC_EINVAL, "the batch runs periodic transverse boundaries only");
    }
    for (int32_t it = 0; it < nsteps; ++it) PICCHK(batch_one_step(b));
    return PIC_OK;
}

pic_status pic_batch_sync(pic_batch* b) {
    if (!b) return PIC_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->m.size(); ++i) PICCHK(bmember(b, (int)i, device_errors(b->m[i])));
    return PIC_OK;
}

pic_status pic_batch_profile_enable(pic_batch* b, int32_t enable) {
    if (!b) return PIC_EINVAL;
    BHIPCHK(b, b->prof.enable(b->stream, enable != 0));
    return PIC_OK;
}

pic_status pic_batch_profile_read(pic_batch* b, pic_profile* out) {
    if (!b || !out) return PIC_EINVAL;
    BHIPCHK(b, b->prof.read(b->stream, out));
    return PIC_OK;
}

const char* pic_batch_last_error(const pic_batch* b) {
    if (!b) return "null batch";
    return b->err.c_str();
}

void pic_batch_destroy(pic_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"
