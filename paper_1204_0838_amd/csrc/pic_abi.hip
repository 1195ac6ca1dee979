// Host side of the C ABI declared in include/pic.h: descriptor validation,
// workspace layout, context state and the launch sequences of each call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

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

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Device workspace carve-up.  Per-particle arrays have max_particles entries;
// species take consecutive sub-ranges of them.
struct Layout {
    size_t acc, jtmp, rho, small, prev_cell, prev_off, alt_cell, alt_off, alt_u, alt_w, alt_id, sort_rank, hist,
        blocks, total;
};

// small block: err flags, per-species counts, reduction results
struct Small {
    int err;
    int pad0;
    int count[kMaxSpecies];
    double red[4];
    unsigned long long live;
    unsigned long long contmax;
    unsigned int jmax;
    int pad1;
};

Layout layout(int64_t ncell, int64_t maxp) {
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
    L.hist = take(((size_t)ncell + 1) * 4);
    L.blocks = take((((size_t)ncell + 1023) / 1024 + 1) * 4 + 4096);
    L.total = o;
    return L;
}

struct Species {
    pic_species_bufs user;   // caller's arrays
    pic_species_bufs cur;    // arrays holding the current data (user's or the workspace copy)
    pic_species_bufs alt;    // the other set
    int64_t base;            // offset into per-particle workspace arrays
    int64_t bound;           // host upper bound of the live count
    bool prev_valid;
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
    Geom g;
    PDCoef pd;
    std::vector<Species> sp;
    int64_t step;
    std::string err;
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
    for (int a = 0; a < 3; ++a)
        if (d->tile[a] < 0 || (d->tile[a] > 0 && d->tile[a] > d->n[a])) return bad("tile larger than the grid");
    if (d->sort_interval < 0) return bad("negative sort interval");
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

SpeciesDev dev_of(const pic_ctx* c, const Species& s) {
    SpeciesDev d;
    d.cell = s.cur.cell;
    for (int a = 0; a < 3; ++a) {
        d.off[a] = s.cur.off[a];
        d.u[a] = s.cur.u[a];
    }
    d.w = s.cur.w;
    d.id = s.cur.id;
    d.qmh = (float)(s.user.q * c->desc.dt / (2.0 * s.user.m));
    d.mq = (float)(-s.user.q);
    return d;
}

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
        if (flags & ERR_OVERFLOW) return fail(c, PIC_EOVERFLOW, "tile or capacity overflow on the device");
    }
    return PIC_OK;
}

pic_status field_update(pic_ctx* c, float* const Juse[3]) {
    FieldPtrs f = fields_of(c);
    const int pd = c->desc.solver == PIC_SOLVER_PD;
    HIPCHK(c, launch_bhalf(c->g, pd, c->pd, f.E, f.B, (float)(0.5 * c->desc.dt), c->stream));
    HIPCHK(c, launch_efull(c->g, f.E, f.B, Juse, c->stream));
    HIPCHK(c, launch_bhalf(c->g, pd, c->pd, f.E, f.B, (float)(0.5 * c->desc.dt), c->stream));
    return PIC_OK;
}

}  // namespace

extern "C" {

size_t pic_workspace_bytes(const pic_grid_desc* desc, int64_t max_particles) {
    if (validate(desc, nullptr, 0) != PIC_OK || max_particles < 0) return 0;
    const int64_t ncell = (int64_t)desc->n[0] * desc->n[1] * desc->n[2];
    return layout(ncell, max_particles > 0 ? max_particles : 1).total;
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
    Layout L = layout(ncell, maxp);
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
    g.dt = (float)desc->dt;
    pd_coefficients(desc, &c->pd);
    hipError_t e = hipMemsetAsync(c->ws + L.acc, 0, 3 * (size_t)ncell * 8, c->stream);
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
    int cnt = (int)n;
    HIPCHK(c, hipMemcpyAsync(&small_of(c)->count[idx], &cnt, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pused += bufs->capacity;
    c->sp.push_back(s);
    if (species_out) *species_out = idx;
    return PIC_OK;
}

pic_status pic_gather_push(pic_ctx* c, int32_t s) {
    pic_status st = check_species(c, s);
    if (st != PIC_OK) return st;
    Species& sp = c->sp[s];
    HIPCHK(c, launch_gather_push(c->g, fields_of(c), dev_of(c, sp), prev_of(c, sp), &small_of(c)->count[s],
                                 (int)sp.bound, &small_of(c)->err, c->stream));
    sp.prev_valid = true;
    return PIC_OK;
}

pic_status pic_deposit(pic_ctx* c, int32_t s) {
    pic_status st = check_species(c, s);
    if (st != PIC_OK) return st;
    Species& sp = c->sp[s];
    if (!sp.prev_valid) return fail(c, PIC_ESTATE, "deposit needs a preceding gather_push");
    HIPCHK(c, launch_deposit(c->g, dev_of(c, sp), prev_of(c, sp), &small_of(c)->count[s], (int)sp.bound, acc_of(c),
                             c->stream));
    double sc[3];
    jscale(c, sc);
    HIPCHK(c, launch_jfinal(c->g, acc_of(c), c->f.J, sc, 0, c->stream));
    return PIC_OK;
}

pic_status pic_field_step(pic_ctx* c) {
    if (!c) return PIC_EINVAL;
    float* Juse[3] = {c->f.J[0], c->f.J[1], c->f.J[2]};
    if (c->desc.jpost == PIC_JPOST_BINOMIAL) {
        float* tmp[3];
        jtmp_of(c, tmp);
        HIPCHK(c, launch_binomial(c->g, c->f.J, tmp, c->stream));
        for (int a = 0; a < 3; ++a)
            HIPCHK(c, hipMemcpyAsync(c->f.J[a], tmp[a], (size_t)c->g.ncell * 4, hipMemcpyDeviceToDevice, c->stream));
    } else if (c->desc.jpost == PIC_JPOST_DENOISER) {
        return fail(c, PIC_EINVAL, "denoiser weights not set");
    }
    pic_status st = field_update(c, Juse);
    if (st != PIC_OK) return st;
    HIPCHK(c, launch_zero_u64(acc_of(c), 3 * (int64_t)c->g.ncell, c->stream));
    c->step += 1;
    return PIC_OK;
}

pic_status pic_step(pic_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return PIC_EINVAL;
    double sc[3];
    jscale(c, sc);
    for (int32_t it = 0; it < nsteps; ++it) {
        for (int32_t s = 0; s < (int32_t)c->sp.size(); ++s) {
            Species& sp = c->sp[s];
            HIPCHK(c, launch_gather_push(c->g, fields_of(c), dev_of(c, sp), prev_of(c, sp), &small_of(c)->count[s],
                                         (int)sp.bound, &small_of(c)->err, c->stream));
            HIPCHK(c, launch_deposit(c->g, dev_of(c, sp), prev_of(c, sp), &small_of(c)->count[s], (int)sp.bound,
                                     acc_of(c), c->stream));
            sp.prev_valid = true;
        }
        float* Juse[3] = {c->f.J[0], c->f.J[1], c->f.J[2]};
        if (c->desc.jpost == PIC_JPOST_BINOMIAL) {
            float* tmp[3];
            jtmp_of(c, tmp);
            HIPCHK(c, launch_jfinal(c->g, acc_of(c), tmp, sc, 1, c->stream));
            HIPCHK(c, launch_binomial(c->g, tmp, c->f.J, c->stream));
        } else if (c->desc.jpost == PIC_JPOST_NONE) {
            HIPCHK(c, launch_jfinal(c->g, acc_of(c), c->f.J, sc, 1, c->stream));
        } else {
            return fail(c, PIC_EINVAL, "denoiser weights not set");
        }
        pic_status st = field_update(c, Juse);
        if (st != PIC_OK) return st;
        c->step += 1;
    }
    return PIC_OK;
}

pic_status pic_sort(pic_ctx* c, int32_t s) {
    pic_status st = check_species(c, s);
    if (st != PIC_OK) return st;
    return fail(c, PIC_EINVAL, "sort not available");
}

pic_status pic_species_view(pic_ctx* c, int32_t s, pic_species_bufs* out, int64_t* n_live) {
    pic_status st = check_species(c, s);
    if (st != PIC_OK) return st;
    int cnt = 0;
    HIPCHK(c, hipMemcpyAsync(&cnt, &small_of(c)->count[s], sizeof(int), hipMemcpyDeviceToHost, c->stream));
    st = device_errors(c);
    if (out) *out = c->sp[s].cur;
    if (n_live) *n_live = cnt;
    return st;
}

pic_status pic_continuity(pic_ctx* c, int32_t s, double* resid, double* max_abs_j) {
    pic_status st = check_species(c, s);
    if (st != PIC_OK) return st;
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
                                c->desc.d[0] / c->desc.d[2], &sm->contmax, c->stream));
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

const char* pic_last_error(const pic_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

void pic_destroy(pic_ctx* c) { delete c; }

}  // extern "C"
