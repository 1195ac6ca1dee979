/*
 * pic_circ.h -- C ABI of the quasi-cylindrical particle-in-cell step with two
 * azimuthal modes (m = 0, 1) in libpic355.so.
 *
 * Section 1 of arXiv:1204.0838 describes the reduced-geometry code it
 * benchmarks against: fields and currents decomposed into poloidal
 * (azimuthal) modes on a radial grid, the macroparticles keeping their full
 * 3D Cartesian motion; Section 3.1 runs it with the two lowest modes and a
 * linearly polarised laser.  This library advances that cycle on one
 * MI355X: gather of both modes at each field component's staggered
 * position, relativistic Boris push and Cartesian move, a charge-conserving
 * deposit of each mode's current, and the per-mode FDTD update of
 * Maxwell's equations in (z, r) with the axis rules that regularity fixes.
 * The paper gives no discretisation; the one here (stated in full beside
 * the FP64 reference of the test suite):
 *
 *   modes     F(r, th, z) = F_0(r, z) + Re(F_1(r, z) exp(-i th))
 *   grid      z nodes i dz (i < nz), r nodes j dr (j < nr), a conducting
 *             wall at r = nr dr; staggering (z, r): E_z (i+1/2, j),
 *             E_r (i, j+1/2), E_th (i, j), B_z (i, j+1/2), B_r (i+1/2, j),
 *             B_th (i+1/2, j+1/2), J like E
 *   shapes    linear in z; in r linear with the correction that makes a
 *             uniform 3D density deposit exactly its value on every node,
 *             the axis node included
 *   deposit   Esirkepov's decomposition of the change of a_i b_j kappa
 *             exp(i m th): each mode's discrete continuity equation holds
 *             exactly off the axis (and on it for m = 0)
 *   axis      m = 0: E_th = B_r = 0, d_t E_z from the flux of B_th through
 *             the cylinder of radius dr/2; m = 1: E_z = 0, d_r B_z and
 *             (1/r) E_z from the odd extension of B_z and E_z
 *
 * Units, errors, streams, ownership and threading are those of pic.h.
 *
 * Field planes: every component of every mode is held in three FP32 planes
 * of nz * nr values (z fastest: index i + nz * j) -- channel 0 the m = 0
 * field, channels 1 and 2 the real and imaginary parts of m = 1.  With a
 * moving window z is a circular buffer (as x in pic.h).
 *
 * Particles use pic_species_bufs with this meaning of its arrays:
 *   cell   iz + nz * jr, iz the storage z cell, jr = floor(r / dr); < 0 removed
 *   off[0] z offset in [0, 1): z = (iz + off[0]) dz (window coordinates
 *          counted from the window origin)
 *   off[1], off[2]  the Cartesian transverse position x, y (c/w_pe)
 *   u[3]   u_x, u_y, u_z (u = gamma v / c)
 *   w      the macroparticle's charge weight: density x volume it stands for
 *   id     tag
 */
#ifndef PIC355_CIRC_H
#define PIC355_CIRC_H

#include "pic.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Grid descriptor.
 *   nz, nr        cells along z (propagation axis) and r; nz >= 16, nr >= 8.
 *   dz, dr, dt    spacings and time step: dt < dz and dt < dr (moves below
 *                 one cell per step) and dt below the grid's Courant limit
 *                 0.95 / sqrt(1/dz^2 + 4/dr^2).
 *   window_period with a moving window (pic_circ_set_window), the window
 *                 moves one cell every window_period steps; c dt = dz /
 *                 window_period is required then (0 = no window).
 *   sort_interval steps between cell sorts in pic_circ_step (0 = 2).
 *   interleave    after a sort, each full block of 64 x interleave particles
 *                 of a tile is stored interleave x 64 transposed, so that at
 *                 interleave particles per cell a wavefront's lanes sit in
 *                 different cells (0 = 32; 1 = plain cell order; at most 64).
 *                 Results do not depend on it.
 *   threads       workgroup size of the fused tile kernel: 256, 512 or 1024
 *                 (0 = 512).  Results do not depend on it. */
typedef struct {
    int32_t nz, nr;
    double dz, dr, dt;
    int32_t window_period;
    int32_t sort_interval;
    int32_t interleave;
    int32_t threads;
} pic_circ_desc;

/* Caller-owned device planes: [component z, r, th][channel m0, Re m1, Im m1]. */
typedef struct {
    float *E[3][3];
    float *B[3][3];
    float *J[3][3];
} pic_circ_fields;

/* Laser on mode 1, linearly polarised along x (Section 3.1):
 * E_x = B_y = e(t - (z - z_src)) exp(-r^2 / waist^2) with e(t) the
 * derivative of the vector potential of pic_laser_desc (a0, omega0, fwhm,
 * t_peak), entering through total-field / scattered-field corrections on
 * the source plane src_z while t <= t_end and the window has not moved. */
typedef struct {
    double a0, omega0, waist, fwhm, t_peak, t_end;
    int32_t src_z;
    int32_t pad_;
} pic_circ_laser;

/* Cold plasma: ppc particles per (z, r) cell in radial cells [0, r_cells),
 * density n(z_lab) 0 before z_start, linear over `ramp`, then n_plateau
 * (lengths in c/w_pe).  Particle (lab cell Z, radial cell j, slot s) draws
 * three uniforms 3c, 3c+1, 3c+2 of the SplitMix64 stream `seed`
 * (c = (Z nr + j) ppc + s; draw k = mix64(seed G + (k + 1) G), top 53 bits):
 * its z offset (rounded toward zero onto 2^-24), r = (j + u) dr and the
 * azimuth 2 pi u; weight n(z_lab) 2 pi r dr dz / ppc; tag c mod 2^31. */
typedef struct {
    double z_start, ramp, n_plateau;
    int32_t ppc;
    int32_t r_cells;
    uint64_t seed;
} pic_circ_plasma;

typedef struct pic_circ_ctx pic_circ_ctx;

/* Validate a descriptor (pure host); message into msg (may be NULL). */
pic_status pic_circ_validate(const pic_circ_desc *desc, char *msg, size_t msg_len);

/* Device workspace for the grid and a total particle capacity (pure host). */
size_t pic_circ_workspace_bytes(const pic_circ_desc *desc, int64_t max_particles);

/* Create a context over caller-owned planes and workspace (256-byte
 * aligned, at least pic_circ_workspace_bytes); stream: the caller's
 * hipStream_t.  Fields are not modified. */
pic_status pic_circ_init(pic_circ_ctx **out, const pic_circ_desc *desc, const pic_circ_fields *fields,
                         void *workspace, size_t workspace_bytes, int64_t max_particles, void *stream);

/* Register a species (host struct copied; arrays hold n valid particles). */
pic_status pic_circ_init_species(pic_circ_ctx *ctx, const pic_species_bufs *bufs, int64_t n, int32_t *species_out);

/* Gather both modes + Boris push + move of one species (x^n, u^{n-1/2} ->
 * x^{n+1}, u^{n+1/2}); keeps x^n for pic_circ_deposit.  Asynchronous. */
pic_status pic_circ_gather_push(pic_circ_ctx *ctx, int32_t species);

/* Charge-conserving deposit of the species' last move into the exact int64
 * accumulator of every mode's current.  Asynchronous. */
pic_status pic_circ_deposit(pic_circ_ctx *ctx, int32_t species);

/* Current read-out (J planes), then B half step, E step, B half step per
 * mode (laser while active), then the window move when due.  Asynchronous. */
pic_status pic_circ_field_step(pic_circ_ctx *ctx);

/* nsteps production steps: periodic cell sort, fused tiled
 * gather+push+deposit of every species, read-out, field update, window.
 * Equal to pic_circ_gather_push + pic_circ_deposit (all species) +
 * pic_circ_field_step per step, bit for bit.  Asynchronous. */
pic_status pic_circ_step(pic_circ_ctx *ctx, int32_t nsteps);

pic_status pic_circ_set_laser(pic_circ_ctx *ctx, const pic_circ_laser *laser);
pic_status pic_circ_set_plasma(pic_circ_ctx *ctx, int32_t species, const pic_circ_plasma *plasma);

/* Load the species' plasma of window z cells [z_begin, z_end) (host-side
 * capacity bound; PIC_ENOMEM beyond it).  Asynchronous. */
pic_status pic_circ_inject_plasma(pic_circ_ctx *ctx, int32_t species, int32_t z_begin, int32_t z_end);

/* Moving window: after every step whose index + 1 >= start_step and
 * (index + 1 - start_step) is a multiple of window_period, the window moves
 * one cell (the leaving plane becomes the zeroed front plane; species with
 * a plasma get the newly covered cell loaded at window cell nz - 3).
 * Particles outside window z cells [2, nz - 3] (after the move) or at
 * r >= (nr - 2) dr are removed after every step (the former are skipped and
 * dropped by the next step; pic_circ_reduce does not count them). */
pic_status pic_circ_set_window(pic_circ_ctx *ctx, int64_t start_step);
pic_status pic_circ_window_state(pic_circ_ctx *ctx, int64_t *shift, int32_t *origin);

/* Current arrays and count of a species (synchronises). */
pic_status pic_circ_species_view(pic_circ_ctx *ctx, int32_t species, pic_species_bufs *out, int64_t *n);

/* FP64 diagnostics: charge sum q w, kinetic energy sum m w (gamma - 1),
 * field energy sum over nodes of V (|F_0|^2 + |F_1|^2 / 2) / 2, max |J| over
 * the nine current planes, live particles, completed steps.  Synchronises. */
pic_status pic_circ_reduce(pic_circ_ctx *ctx, pic_diag *out);

pic_status pic_circ_sync(pic_circ_ctx *ctx);

/* Phase timing as pic_profile_enable / pic_profile_read (sort, tile, rest,
 * read-out, field, window). */
pic_status pic_circ_profile_enable(pic_circ_ctx *ctx, int32_t enable);
pic_status pic_circ_profile_read(pic_circ_ctx *ctx, pic_profile *out);

const char *pic_circ_last_error(const pic_circ_ctx *ctx);
void pic_circ_destroy(pic_circ_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PIC355_CIRC_H */
