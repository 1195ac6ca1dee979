// Host side of the quasi-cylindrical C ABI (include/pic_circ.h): descriptor
// validation, workspace layout, context state and the launch sequence of a
// step.  The cell sort is the Cartesian library's counting sort run on a
// (nz, nr, 1) grid, so particles of one (z, r) tile are contiguous.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "pic_circ.h"
#include "pic_circ_internal.h"

using namespace pic;

namespace {

constexpr int kCircMaxSpecies = 8;
constexpr size_t kAlignC = 256;
constexpr int kKill = 2;   // window z cells kept: [kKill, nz - 1 - kKill]
constexpr int kWall = 2;   // particles at r >= (nr - kWall) dr are removed

size_t alignc(size_t v) { return (v + kAlignC - 1) / kAlignC * kAlignC; }

struct CSmall {
    int err;
    int pad0;
    int count[kCircMaxSpecies];
    int sorted[kCircMaxSpecies];
    int rest_n[kCircMaxSpecies];
    double red[4];
    unsigned long long live;
    unsigned int jmax;
    int pad1;
};

struct CLayout {
    size_t acc, small, prev_cell, prev_off, alt_cell, alt_off, alt_u, alt_w, alt_id, rank, hist, sums, toff,
        toff_stride, total;
};

TileGeom circ_tiles(const pic_circ_desc* d) {
    TileGeom t;
    t.T[0] = circ_tile_z() < d->nz ? circ_tile_z() : d->nz;
    t.T[1] = circ_tile_r() < d->nr ? circ_tile_r() : d->nr;
    t.T[2] = 1;
    t.nt[0] = (d->nz + t.T[0] - 1) / t.T[0];
    t.nt[1] = (d->nr + t.T[1] - 1) / t.T[1];
    t.nt[2] = 1;
    t.ntiles = t.nt[0] * t.nt[1];
    t.tcells = t.T[0] * t.T[1];
    return t;
}

CLayout clayout(const pic_circ_desc* d, int64_t maxp) {
    const int64_t ncell = (int64_t)d->nz * d->nr;
    const TileGeom t = circ_tiles(d);
    const int64_t nkeys = (int64_t)t.ntiles * t.tcells;
    CLayout L;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t at = o;
        o = alignc(o + b);
        return at;
    };
    L.acc = take((size_t)kCircChannels * ncell * 8);
    L.small = take(sizeof(CSmall));
    L.prev_cell = take((size_t)maxp * 4);
    L.prev_off = take(3 * alignc((size_t)maxp * 4));
    L.alt_cell = take((size_t)maxp * 4);
    L.alt_off = take(3 * alignc((size_t)maxp * 4));
    L.alt_u = take(3 * alignc((size_t)maxp * 4));
    L.alt_w = take((size_t)maxp * 4);
    L.alt_id = take((size_t)maxp * 4);
    L.rank = take((size_t)maxp * 4);
    L.hist = take(((size_t)nkeys + 1) * 4);
    L.sums = take((((size_t)nkeys + 1 + 1023) / 1024 + 1) * 4);
    L.toff_stride = alignc(((size_t)t.ntiles + 1) * 4);
    L.toff = take(kCircMaxSpecies * L.toff_stride);
    L.total = o;
    return L;
}

pic_status cvalidate(const pic_circ_desc* d, char* msg, size_t len) {
    auto bad = [&](const char* why) {
        if (msg && len) snprintf(msg, len, "%s", why);
        return PIC_EINVAL;
    };
    if (!d) return bad("null descriptor");
    if (d->nz < 16 || d->nr < 8) return bad("the grid needs nz >= 16 and nr >= 8");
    if ((int64_t)d->nz * d->nr >= (1ll << 30)) return bad("grid exceeds 2^30 cells");
    if (!(d->dz > 0) || !(d->dr > 0) || !(d->dt > 0) || !isfinite(d->dz) || !isfinite(d->dr) || !isfinite(d->dt))
        return bad("spacings and time step must be positive and finite");
    if (!(d->dt < d->dz) || !(d->dt < d->dr)) return bad("dt must be below dz and dr");
    if (!(d->dt <= 0.95 / sqrt(1.0 / (d->dz * d->dz) + 4.0 / (d->dr * d->dr))))
        return bad("time step above the cylindrical Courant bound 0.95/sqrt(1/dz^2 + 4/dr^2)");
    if (d->window_period < 0 || d->sort_interval < 0) return bad("negative window period or sort interval");
    if (d->interleave < 0 || d->interleave > 64) return bad("interleave outside [0, 64]");
    if (d->threads != 0 && d->threads != 256 && d->threads != 512 && d->threads != 1024)
        return bad("threads per tile must be 0, 256, 512 or 1024");
    if (d->window_period > 0 && fabs(d->dt * d->window_period - d->dz) > 1e-12 * d->dz)
        return bad("a window moving one cell every window_period steps needs c dt = dz / window_period");
    if (msg && len) msg[0] = 0;
    return PIC_OK;
}

struct CSpecies {
    pic_species_bufs user, cur, alt;
    int64_t base, bound, sort_step;
    bool sorted, prev_valid;
};

enum { CP_SORT, CP_TILE, CP_REST, CP_JPOST, CP_FIELD, CP_WINDOW, CP_COUNT };

}  // namespace

struct pic_circ_ctx {
    pic_circ_desc desc;
    pic_circ_fields f;
    hipStream_t stream;
    char* ws;
    int64_t maxp, pused;
    CLayout L;
    TileGeom t;
    CircGeom g;
    std::vector<CSpecies> sp;
    int64_t step = 0;
    std::string err;
    bool has_laser = false;
    pic_circ_laser laser;
    int64_t window_start = INT64_MAX;
    int64_t shift = 0;
    bool has_plasma[kCircMaxSpecies] = {};
    pic_circ_plasma plasma[kCircMaxSpecies];
    // phase timing
    bool prof_on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Mark {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    int64_t psteps = 0, psorts = 0, ptiles = 0;
    ~pic_circ_ctx() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

namespace {

pic_status cfail(pic_circ_ctx* c, pic_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define CHIP(ctx, expr)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return cfail(ctx, PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define CCHK(expr)                   \
    do {                             \
        pic_status s_ = (expr);      \
        if (s_ != PIC_OK) return s_; \
    } while (0)

CSmall* csmall(pic_circ_ctx* c) { return reinterpret_cast<CSmall*>(c->ws + c->L.small); }
unsigned long long* cacc(pic_circ_ctx* c) { return reinterpret_cast<unsigned long long*>(c->ws + c->L.acc); }
int* ctoff(pic_circ_ctx* c, int s) { return reinterpret_cast<int*>(c->ws + c->L.toff + (size_t)s * c->L.toff_stride); }

SpeciesDev cdev(const pic_circ_ctx* c, const CSpecies& s, const pic_species_bufs& b) {
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

PrevDev cprev(pic_circ_ctx* c, const CSpecies& s) {
    PrevDev p;
    p.cell = reinterpret_cast<int*>(c->ws + c->L.prev_cell) + s.base;
    const size_t stride = alignc((size_t)c->maxp * 4);
    for (int a = 0; a < 3; ++a) p.off[a] = reinterpret_cast<float*>(c->ws + c->L.prev_off + a * stride) + s.base;
    return p;
}

CircFields cfields(const pic_circ_ctx* c) {
    CircFields F;
    for (int comp = 0; comp < 3; ++comp)
        for (int ch = 0; ch < 3; ++ch) {
            F.F[0][comp][ch] = c->f.E[comp][ch];
            F.F[1][comp][ch] = c->f.B[comp][ch];
        }
    return F;
}

void cfield_planes(const pic_circ_ctx* c, float* F[2][3][3]) {
    for (int comp = 0; comp < 3; ++comp)
        for (int ch = 0; ch < 3; ++ch) {
            F[0][comp][ch] = c->f.E[comp][ch];
            F[1][comp][ch] = c->f.B[comp][ch];
        }
}

void cj(const pic_circ_ctx* c, float* J[9]) {
    for (int comp = 0; comp < 3; ++comp)
        for (int ch = 0; ch < 3; ++ch) J[comp * 3 + ch] = c->f.J[comp][ch];
}

// Geometry of the (nz, nr, 1) grid seen by the Cartesian sort.
Geom sort_geom(const pic_circ_ctx* c) {
    Geom g;
    memset(&g, 0, sizeof g);
    g.n[0] = c->desc.nz;
    g.n[1] = c->desc.nr;
    g.n[2] = 1;
    g.nxy = c->desc.nz * c->desc.nr;
    g.ncell = g.nxy;
    g.window = c->g.window;
    g.origin = c->g.origin;
    g.kill_lo = kKill;
    g.kill_hi = kKill;
    return g;
}

pic_status cmark(pic_circ_ctx* c, hipEvent_t* ev) {
    *ev = nullptr;
    if (!c->prof_on) return PIC_OK;
    if (c->used == c->pool.size()) {
        hipEvent_t e;
        CHIP(c, hipEventCreate(&e));
        c->pool.push_back(e);
    }
    *ev = c->pool[c->used++];
    CHIP(c, hipEventRecord(*ev, c->stream));
    return PIC_OK;
}

pic_status cend(pic_circ_ctx* c, int phase, hipEvent_t start) {
    if (!c->prof_on || !start) return PIC_OK;
    hipEvent_t e;
    CCHK(cmark(c, &e));
    c->marks.push_back({phase, start, e});
    return PIC_OK;
}

pic_status cdevice_errors(pic_circ_ctx* c) {
    int flags = 0;
    CHIP(c, hipMemcpyAsync(&flags, &csmall(c)->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CHIP(c, hipStreamSynchronize(c->stream));
    if (flags) {
        CHIP(c, hipMemsetAsync(&csmall(c)->err, 0, sizeof(int), c->stream));
        if (flags & ERR_NONFINITE) return cfail(c, PIC_ENONFINITE, "non-finite momentum on the device");
        if (flags & ERR_CFL) return cfail(c, PIC_ECFL, "a particle moved one cell or more along z in a step");
        if (flags & ERR_OVERFLOW) return cfail(c, PIC_EOVERFLOW, "particle capacity exceeded on the device");
    }
    return PIC_OK;
}

pic_status ccheck_species(pic_circ_ctx* c, int32_t s) {
    if (!c) return PIC_EINVAL;
    if (s < 0 || s >= (int32_t)c->sp.size()) return cfail(c, PIC_EINVAL, "no species %d", s);
    return PIC_OK;
}

// e(t) of the laser (the time derivative of -A of pic_laser_desc's pulse)
double claser_e(const pic_circ_laser& L, double t) {
    const double tau = t - L.t_peak;
    const double k = 2.0 * log(2.0) / (L.fwhm * L.fwhm);
    const double env = exp(-k * tau * tau);
    const double denv = -2.0 * k * tau * env;
    const double ph = L.omega0 * tau;
    return L.a0 * (env * L.omega0 * sin(ph) - denv * cos(ph));
}

pic_status cfield_update(pic_circ_ctx* c) {
    float* F[2][3][3];
    cfield_planes(c, F);
    float* J[9];
    cj(c, J);
    const double dt = c->desc.dt, dz = c->desc.dz, t = c->step * dt;
    const bool laser = c->has_laser && c->shift == 0 && t <= c->laser.t_end;
    const double iw2 = laser ? 1.0 / (c->laser.waist * c->laser.waist) : 0.0;
    const int src = laser ? c->laser.src_z : 0;
    const int bplane = (src - 1 + (c->g.window ? c->g.origin : 0)) % c->desc.nz;
    const int eplane = (src + (c->g.window ? c->g.origin : 0)) % c->desc.nz;
    CHIP(c, launch_circ_bhalf(c->g, F, (float)(0.5 * dt), c->stream));
    if (laser) CHIP(c, launch_circ_laser(c->g, F, bplane, 0, 0.5 * dt * claser_e(c->laser, t) / dz, iw2, c->stream));
    CHIP(c, launch_circ_efull(c->g, F, J, c->stream));
    if (laser)
        CHIP(c, launch_circ_laser(c->g, F, eplane, 1, dt * claser_e(c->laser, t + 0.5 * dt + 0.5 * dz) / dz, iw2,
                                  c->stream));
    CHIP(c, launch_circ_bhalf(c->g, F, (float)(0.5 * dt), c->stream));
    if (laser)
        CHIP(c, launch_circ_laser(c->g, F, bplane, 0, 0.5 * dt * claser_e(c->laser, t + dt) / dz, iw2, c->stream));
    return PIC_OK;
}

pic_status cinject(pic_circ_ctx* c, int32_t s, int32_t zb, int32_t ze) {
    CSpecies& sp = c->sp[s];
    const pic_circ_plasma& P = c->plasma[s];
    const int64_t most = (int64_t)(ze - zb) * P.r_cells * P.ppc;
    if (most <= 0) return PIC_OK;
    if (sp.bound + most > sp.user.capacity) {
        int v = 0;
        CHIP(c, hipMemcpyAsync(&v, &csmall(c)->count[s], sizeof(int), hipMemcpyDeviceToHost, c->stream));
        CHIP(c, hipStreamSynchronize(c->stream));
        sp.bound = v;
        if (sp.bound + most > sp.user.capacity)
            return cfail(c, PIC_ENOMEM, "species %d: %lld particles plus up to %lld injected exceed capacity %lld", s,
                         (long long)sp.bound, (long long)most, (long long)sp.user.capacity);
    }
    CHIP(c, launch_circ_inject(c->g, cdev(c, sp, sp.cur), (long long)c->shift, zb, ze, P.r_cells, P.ppc, P.seed,
                               P.z_start, P.ramp, P.n_plateau, c->desc.dz, c->desc.dr, &csmall(c)->count[s],
                               (int)sp.user.capacity, &csmall(c)->err, c->stream));
    sp.bound += most;
    return PIC_OK;
}

pic_status cend_step(pic_circ_ctx* c) {
    c->step += 1;
    if (c->prof_on) c->psteps += 1;
    if (!c->g.window || c->step < c->window_start) return PIC_OK;
    if ((c->step - c->window_start) % c->desc.window_period != 0) return PIC_OK;
    hipEvent_t t0;
    CCHK(cmark(c, &t0));
    float* F[2][3][3];
    cfield_planes(c, F);
    CHIP(c, launch_circ_clear_plane(c->g, F, c->g.origin, c->stream));
    c->g.origin = c->g.origin + 1 == c->desc.nz ? 0 : c->g.origin + 1;
    c->shift += 1;
    const int slab = c->desc.nz - 1 - kKill;
    for (int32_t s = 0; s < (int32_t)c->sp.size(); ++s)
        if (c->has_plasma[s]) CCHK(cinject(c, s, slab, slab + 1));
    return cend(c, CP_WINDOW, t0);
}

// read-out of the accumulated current, field update, window
pic_status cfinish_step(pic_circ_ctx* c) {
    hipEvent_t t0, t1;
    CCHK(cmark(c, &t0));
    float* J[9];
    cj(c, J);
    CHIP(c, launch_circ_jfinal(c->g, cacc(c), J, 1, c->stream));
    CCHK(cend(c, CP_JPOST, t0));
    CCHK(cmark(c, &t1));
    CCHK(cfield_update(c));
    CCHK(cend(c, CP_FIELD, t1));
    return cend_step(c);
}

}  // namespace

extern "C" {

pic_status pic_circ_validate(const pic_circ_desc* desc, char* msg, size_t msg_len) {
    return cvalidate(desc, msg, msg_len);
}

size_t pic_circ_workspace_bytes(const pic_circ_desc* desc, int64_t max_particles) {
    if (cvalidate(desc, nullptr, 0) != PIC_OK || max_particles < 0) return 0;
    return clayout(desc, max_particles > 0 ? max_particles : 1).total;
}

pic_status pic_circ_init(pic_circ_ctx** out, const pic_circ_desc* desc, const pic_circ_fields* fields,
                         void* workspace, size_t workspace_bytes, int64_t max_particles, void* stream) {
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    pic_status st = cvalidate(desc, nullptr, 0);
    if (st != PIC_OK) return st;
    if (!fields || !workspace || max_particles < 0) return PIC_EINVAL;
    for (int a = 0; a < 3; ++a)
        for (int ch = 0; ch < 3; ++ch)
            if (!fields->E[a][ch] || !fields->B[a][ch] || !fields->J[a][ch]) return PIC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlignC - 1)) != 0) return PIC_EINVAL;
    const int64_t maxp = max_particles > 0 ? max_particles : 1;
    CLayout L = clayout(desc, maxp);
    if (workspace_bytes < L.total) return PIC_ENOMEM;
    if (circ_tile_lds() > 160 * 1024) return PIC_EINVAL;
    pic_circ_ctx* c = new (std::nothrow) pic_circ_ctx();
    if (!c) return PIC_ENOMEM;
    c->desc = *desc;
    if (c->desc.sort_interval == 0) c->desc.sort_interval = 2;
    if (c->desc.interleave == 0) c->desc.interleave = 32;
    if (c->desc.threads == 0) c->desc.threads = 512;
    c->f = *fields;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    c->ws = reinterpret_cast<char*>(workspace);
    c->maxp = maxp;
    c->pused = 0;
    c->L = L;
    c->t = circ_tiles(desc);
    CircGeom& g = c->g;
    g.nz = desc->nz;
    g.nr = desc->nr;
    g.ncell = desc->nz * desc->nr;
    g.window = desc->window_period > 0;
    g.origin = 0;
    g.kill = g.window ? kKill : 0;
    g.wall = kWall;
    g.dz = (float)desc->dz;
    g.dr = (float)desc->dr;
    g.dt = (float)desc->dt;
    g.inv_dz = (float)(1.0 / desc->dz);
    g.inv_dr = (float)(1.0 / desc->dr);
    g.dtdz = (float)(desc->dt / desc->dz);
    hipError_t e = hipMemsetAsync(c->ws + L.acc, 0, (size_t)kCircChannels * g.ncell * 8, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.small, 0, sizeof(CSmall), c->stream);
    if (e != hipSuccess) {
        delete c;
        return PIC_EDEVICE;
    }
    *out = c;
    return PIC_OK;
}

pic_status pic_circ_init_species(pic_circ_ctx* c, const pic_species_bufs* bufs, int64_t n, int32_t* species_out) {
    if (!c || !bufs) return PIC_EINVAL;
    if ((int)c->sp.size() >= kCircMaxSpecies) return cfail(c, PIC_EINVAL, "at most %d species", kCircMaxSpecies);
    if (!bufs->cell || !bufs->w || !bufs->id) return cfail(c, PIC_EINVAL, "null particle array");
    for (int a = 0; a < 3; ++a)
        if (!bufs->off[a] || !bufs->u[a]) return cfail(c, PIC_EINVAL, "null particle array");
    if (!(bufs->m > 0.0) || !isfinite(bufs->q)) return cfail(c, PIC_EINVAL, "invalid charge or mass");
    if (n < 0 || n > bufs->capacity || bufs->capacity >= (1ll << 31))
        return cfail(c, PIC_EINVAL, "particle count outside [0, capacity] or capacity above 2^31");
    if (c->pused + bufs->capacity > c->maxp)
        return cfail(c, PIC_ENOMEM, "workspace sized for %lld particles", (long long)c->maxp);
    CSpecies s;
    s.user = *bufs;
    s.cur = *bufs;
    s.base = c->pused;
    s.bound = n;
    s.sort_step = 0;
    s.sorted = false;
    s.prev_valid = false;
    const size_t stride = alignc((size_t)c->maxp * 4);
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
    CHIP(c, hipMemcpyAsync(&csmall(c)->count[idx], &cnt[0], sizeof(int), hipMemcpyHostToDevice, c->stream));
    CHIP(c, hipMemcpyAsync(&csmall(c)->sorted[idx], &cnt[1], sizeof(int), hipMemcpyHostToDevice, c->stream));
    CHIP(c, hipStreamSynchronize(c->stream));
    c->pused += bufs->capacity;
    c->sp.push_back(s);
    if (species_out) *species_out = idx;
    return PIC_OK;
}

pic_status pic_circ_gather_push(pic_circ_ctx* c, int32_t s) {
    CCHK(ccheck_species(c, s));
    CSpecies& sp = c->sp[s];
    CHIP(c, launch_circ_gather_push(c->g, cfields(c), cdev(c, sp, sp.cur), cprev(c, sp), &csmall(c)->count[s],
                                    (int)sp.bound, &csmall(c)->err, c->stream));
    sp.prev_valid = true;
    return PIC_OK;
}

pic_status pic_circ_deposit(pic_circ_ctx* c, int32_t s) {
    CCHK(ccheck_species(c, s));
    CSpecies& sp = c->sp[s];
    if (!sp.prev_valid) return cfail(c, PIC_ESTATE, "deposit needs a preceding gather_push");
    CHIP(c, launch_circ_deposit(c->g, cdev(c, sp, sp.cur), cprev(c, sp), &csmall(c)->count[s], (int)sp.bound,
                                (float)sp.user.q, cacc(c), c->stream));
    sp.prev_valid = false;
    return PIC_OK;
}

pic_status pic_circ_field_step(pic_circ_ctx* c) {
    if (!c) return PIC_EINVAL;
    return cfinish_step(c);
}

pic_status pic_circ_step(pic_circ_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return PIC_EINVAL;
    for (int32_t it = 0; it < nsteps; ++it) {
        for (int32_t s = 0; s < (int32_t)c->sp.size(); ++s) {
            CSpecies& sp = c->sp[s];
            if (sp.bound == 0) continue;
            CSmall* sm = csmall(c);
            hipEvent_t t0, t1, t2;
            if (!sp.sorted || c->step - sp.sort_step >= c->desc.sort_interval) {
                CCHK(cmark(c, &t0));
                int* rank = reinterpret_cast<int*>(c->ws + c->L.rank) + sp.base;
                CHIP(c, launch_sort(sort_geom(c), c->t, cdev(c, sp, sp.cur), cdev(c, sp, sp.alt), &sm->count[s],
                                    &sm->sorted[s], (int)sp.bound, reinterpret_cast<int*>(c->ws + c->L.hist), rank,
                                    reinterpret_cast<int*>(c->ws + c->L.sums), nullptr, nullptr, c->desc.interleave, ctoff(c, s),
                                    true, false,
                                    c->stream));
                std::swap(sp.cur, sp.alt);
                sp.sorted = true;
                sp.sort_step = c->step;
                CCHK(cend(c, CP_SORT, t0));
                if (c->prof_on) c->psorts += 1;
            }
            int* rest_idx = reinterpret_cast<int*>(c->ws + c->L.rank) + sp.base;
            CCHK(cmark(c, &t1));
            CHIP(c, launch_circ_tile(c->g, cfields(c), cdev(c, sp, sp.cur), ctoff(c, s), c->t.nt[0], c->t.ntiles,
                                     cacc(c), &sm->err, &sm->rest_n[s], rest_idx, c->desc.threads, c->stream));
            CCHK(cend(c, CP_TILE, t1));
            if (c->prof_on) c->ptiles += 1;
            CCHK(cmark(c, &t2));
            CHIP(c, launch_circ_rest(c->g, cfields(c), cdev(c, sp, sp.cur), &sm->sorted[s], &sm->count[s],
                                     &sm->rest_n[s], rest_idx, (int)sp.bound, cacc(c), &sm->err, c->stream));
            CCHK(cend(c, CP_REST, t2));
            sp.prev_valid = false;
        }
        CCHK(cfinish_step(c));
    }
    return PIC_OK;
}

pic_status pic_circ_set_laser(pic_circ_ctx* c, const pic_circ_laser* L) {
    if (!c) return PIC_EINVAL;
    if (!L) {
        c->has_laser = false;
        return PIC_OK;
    }
    if (L->src_z < 1 || L->src_z >= c->desc.nz - 1) return cfail(c, PIC_EINVAL, "laser source plane outside [1, nz-1)");
    if (!(L->fwhm > 0) || !(L->waist > 0) || !isfinite(L->a0) || !isfinite(L->omega0) || !isfinite(L->t_peak) ||
        !isfinite(L->t_end))
        return cfail(c, PIC_EINVAL, "invalid laser parameters");
    if (c->g.window && c->window_start != INT64_MAX && L->t_end > c->window_start * c->desc.dt)
        return cfail(c, PIC_EINVAL, "the window would move while the laser source is active");
    c->laser = *L;
    c->has_laser = true;
    return PIC_OK;
}

pic_status pic_circ_set_plasma(pic_circ_ctx* c, int32_t s, const pic_circ_plasma* P) {
    CCHK(ccheck_species(c, s));
    if (!P) {
        c->has_plasma[s] = false;
        return PIC_OK;
    }
    if (P->ppc < 1 || P->ppc > 1024) return cfail(c, PIC_EINVAL, "particles per cell outside 1..1024");
    if (P->r_cells < 1 || P->r_cells > c->desc.nr - kWall)
        return cfail(c, PIC_EINVAL, "plasma radial cells outside 1..nr-2");
    if (!(P->ramp >= 0) || !isfinite(P->z_start) || !(P->n_plateau >= 0) || !isfinite(P->n_plateau))
        return cfail(c, PIC_EINVAL, "invalid plasma profile");
    c->plasma[s] = *P;
    c->has_plasma[s] = true;
    return PIC_OK;
}

pic_status pic_circ_inject_plasma(pic_circ_ctx* c, int32_t s, int32_t zb, int32_t ze) {
    CCHK(ccheck_species(c, s));
    if (!c->has_plasma[s]) return cfail(c, PIC_ESTATE, "species %d has no plasma profile", s);
    if (zb < 0 || ze > c->desc.nz || zb > ze) return cfail(c, PIC_EINVAL, "slab outside the grid");
    return cinject(c, s, zb, ze);
}

pic_status pic_circ_set_window(pic_circ_ctx* c, int64_t start_step) {
    if (!c) return PIC_EINVAL;
    if (!c->g.window) return cfail(c, PIC_ESTATE, "the descriptor has no window period");
    if (start_step < 0) return cfail(c, PIC_EINVAL, "negative start step");
    if (c->has_laser && c->laser.t_end > start_step * c->desc.dt)
        return cfail(c, PIC_EINVAL, "the window would move while the laser source is active");
    c->window_start = start_step;
    return PIC_OK;
}

pic_status pic_circ_window_state(pic_circ_ctx* c, int64_t* shift, int32_t* origin) {
    if (!c) return PIC_EINVAL;
    if (shift) *shift = c->shift;
    if (origin) *origin = c->g.origin;
    return PIC_OK;
}

pic_status pic_circ_species_view(pic_circ_ctx* c, int32_t s, pic_species_bufs* out, int64_t* n) {
    CCHK(ccheck_species(c, s));
    int cnt = 0;
    CHIP(c, hipMemcpyAsync(&cnt, &csmall(c)->count[s], sizeof(int), hipMemcpyDeviceToHost, c->stream));
    pic_status st = cdevice_errors(c);
    if (out) *out = c->sp[s].cur;
    if (n) *n = cnt;
    return st;
}

pic_status pic_circ_reduce(pic_circ_ctx* c, pic_diag* out) {
    if (!c || !out) return PIC_EINVAL;
    CSmall* sm = csmall(c);
    CHIP(c, hipMemsetAsync(sm->red, 0, sizeof sm->red, c->stream));
    CHIP(c, hipMemsetAsync(&sm->live, 0, 8, c->stream));
    CHIP(c, hipMemsetAsync(&sm->jmax, 0, 4, c->stream));
    std::vector<SpeciesDev> sd;
    std::vector<const int*> cnt;
    std::vector<double> q, m;
    std::vector<int> mc;
    for (int32_t s = 0; s < (int32_t)c->sp.size(); ++s) {
        CSpecies& sp = c->sp[s];
        sd.push_back(cdev(c, sp, sp.cur));
        cnt.push_back(&sm->count[s]);
        q.push_back(sp.user.q);
        m.push_back(sp.user.m);
        mc.push_back((int)sp.bound);
    }
    float* J[9];
    cj(c, J);
    CHIP(c, launch_circ_diag(c->g, cfields(c), J, sd.data(), cnt.data(), q.data(), m.data(), mc.data(),
                             (int)sd.size(), sm->red, &sm->live, &sm->jmax, c->stream));
    double red[4];
    unsigned long long live = 0;
    unsigned int jm = 0;
    CHIP(c, hipMemcpyAsync(red, sm->red, sizeof red, hipMemcpyDeviceToHost, c->stream));
    CHIP(c, hipMemcpyAsync(&live, &sm->live, 8, hipMemcpyDeviceToHost, c->stream));
    CHIP(c, hipMemcpyAsync(&jm, &sm->jmax, 4, hipMemcpyDeviceToHost, c->stream));
    CHIP(c, hipStreamSynchronize(c->stream));
    float j;
    memcpy(&j, &jm, 4);
    out->charge = red[0];
    out->e_kin = red[1];
    out->e_field = red[2];
    out->max_abs_J = j;
    out->n_particles = (int64_t)live;
    out->step = c->step;
    return cdevice_errors(c);
}

pic_status pic_circ_sync(pic_circ_ctx* c) {
    if (!c) return PIC_EINVAL;
    CHIP(c, hipStreamSynchronize(c->stream));
    return cdevice_errors(c);
}

pic_status pic_circ_profile_enable(pic_circ_ctx* c, int32_t enable) {
    if (!c) return PIC_EINVAL;
    if (enable) {
        CHIP(c, hipStreamSynchronize(c->stream));
        c->marks.clear();
        c->used = 0;
        c->psteps = c->psorts = c->ptiles = 0;
    }
    c->prof_on = enable != 0;
    return PIC_OK;
}

pic_status pic_circ_profile_read(pic_circ_ctx* c, pic_profile* out) {
    if (!c || !out) return PIC_EINVAL;
    CHIP(c, hipStreamSynchronize(c->stream));
    double ms[CP_COUNT] = {0, 0, 0, 0, 0, 0};
    for (const auto& mk : c->marks) {
        float t = 0.0f;
        CHIP(c, hipEventElapsedTime(&t, mk.a, mk.b));
        ms[mk.phase] += t;
    }
    out->sort_ms = ms[CP_SORT];
    out->tile_ms = ms[CP_TILE];
    out->loose_ms = ms[CP_REST];
    out->jpost_ms = ms[CP_JPOST];
    out->field_ms = ms[CP_FIELD];
    out->window_ms = ms[CP_WINDOW];
    out->steps = c->psteps;
    out->sorts = c->psorts;
    out->tile_launches = c->ptiles;
    return PIC_OK;
}

const char* pic_circ_last_error(const pic_circ_ctx* c) { return c ? c->err.c_str() : "null context"; }

void pic_circ_destroy(pic_circ_ctx* c) { delete c; }

}  // extern "C"
