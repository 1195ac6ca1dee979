/*
 * pic.h -- C ABI of the MI355X particle-in-cell library (libpic355.so).
 *
 * The library advances the explicit electromagnetic PIC cycle of
 * arXiv:1204.0838 (Section 1: fields on a grid, macroparticles in continuous
 * phase space; Section 2, eq. 2.1: D_t B = -curl' E, D_t E = c^2 curl B - J/eps0)
 * on one AMD Instinct MI355X (gfx950):
 *
 *   cubic B-spline gather of E, B (third-order shapes, Sections 1 and 3.1)
 *   -> relativistic Boris push -> move -> charge-conserving (Esirkepov) cubic
 *   deposit of J -> optional J filter -> FDTD update in Yee form (curl' = curl,
 *   Section 1) or perfect-dispersion form (curl' with the transverse
 *   smoothing stencils S_x, S_y, S_z of Section 2).
 *
 * Units are plasma-normalised (the w_pe of Section 1): lengths c/w_pe,
 * times 1/w_pe, momenta u = gamma v / c, fields m_e c w_pe / e, densities n0;
 * so c = eps0 = 1.  Electrons have q = -1, m = 1.  Ions are an immobile
 * neutralising background and are not represented.
 *
 * Memory ownership: every device buffer (fields, particles, workspace) is
 * allocated by the caller (e.g. PyTorch-ROCm tensors) and passed as a raw
 * device pointer; the library stores the pointers and never allocates or
 * frees device memory.  Host pointers are marked "host".
 *
 * Streams: all calls enqueue asynchronously on the caller's HIP stream given
 * to pic_init_grid, except those documented as synchronising.
 *
 * Errors: every call returns pic_status (0 = OK, < 0 = error) and never
 * throws.  The context keeps a sticky error whose text pic_last_error
 * returns.  Device-side conditions (a particle moving one cell or more per
 * step, a non-finite momentum, a tile overflow) set a device flag which the
 * next synchronising call (pic_sync, pic_reduce, pic_species_view) reports.
 *
 * Threading: one context per host thread; calls on one context are not
 * re-entrant.
 *
 * Field layout: each of the nine component arrays E[3], B[3], J[3] is a dense
 * FP32 array of n[0]*n[1]*n[2] values, x fastest: index(i,j,k) =
 * i + n0*(j + n1*k).  Yee staggering: index (i,j,k) holds E_x(i+1/2,j,k),
 * E_y(i,j+1/2,k), E_z(i,j,k+1/2), B_x(i,j+1/2,k+1/2), B_y(i+1/2,j,k+1/2),
 * B_z(i+1/2,j+1/2,k), J like E.  y and z are periodic.  x is periodic, or
 * (moving window) a circular buffer whose window origin advances one cell per
 * shift; the two planes where the window ends meet see zero fields beyond.
 *
 * Particle layout (structure of arrays, one entry per macroparticle):
 *   cell  int32   linear cell index i + n0*(j + n1*k) (storage coordinates);
 *                 a negative value marks a removed particle
 *   off   float[3] in-cell offsets in [0, 1): position = (i + off_x) dx, ...
 *   u     float[3] u = gamma v / c
 *   w     float   density weight n/ppc (charge per cell volume q*w)
 *   id    int32   caller's tag, carried through sorting
 */
#ifndef PIC355_H
#define PIC355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,     /* invalid argument or descriptor */
    PIC_ENOMEM = -2,     /* workspace or particle capacity too small */
    PIC_EDEVICE = -3,    /* a HIP runtime call failed */
    PIC_EOVERFLOW = -4,  /* tile / capacity overflow detected on the device */
    PIC_ENONFINITE = -5, /* non-finite momentum detected on the device */
    PIC_ECFL = -6,       /* a particle moved >= 1 cell in a step, or the time step breaks stability */
    PIC_ESTATE = -7      /* call out of order (e.g. deposit before gather_push) */
} pic_status;

enum { PIC_SOLVER_YEE = 0, PIC_SOLVER_PD = 1 };
enum { PIC_BC_PERIODIC = 0, PIC_BC_MOVING_WINDOW = 1 };
enum { PIC_JPOST_NONE = 0, PIC_JPOST_BINOMIAL = 1, PIC_JPOST_DENOISER = 2 };

/* Grid and solver descriptor.
 *   n[3], d[3]   cells and cell sizes; every n >= 4.
 *   dt           time step.  Yee: must satisfy the 3D Courant limit
 *                dt < 1/sqrt(sum 1/d^2).  PD (Section 2): requires
 *                d[0] <= d[1], d[2] (the paper's only constraint) and
 *                dt <= d[0] (c dt = dx gives no axial dispersion).
 *   solver       PIC_SOLVER_YEE or PIC_SOLVER_PD.
 *   pd_variant   PD stencil coefficients: 0 = with corner weights,
 *                1 = corner weights zero.
 *   bc_x         PIC_BC_PERIODIC or PIC_BC_MOVING_WINDOW.
 *   jpost        current post-processing before the field update.
 *   tile[3]      cells per particle tile of the fused step, 3..16 per axis
 *                (0 = default 8; clamped to the grid).
 *   sort_interval steps between cell sorts in pic_step (0 = default 2).
 *   guard        cells a particle may drift out of its tile and still be
 *                handled in LDS (0..3; a negative value selects the
 *                default 1); beyond it the fused step uses global memory
 *                for that particle.  The tile's LDS footprint
 *                24 B x PJ x (Tz + 2 guard + 5) + 24 B x PF x (Tz + 2 guard + 4)
 *                must fit in 160 KiB, where the z-plane sizes
 *                PJ = (Tx + 2 guard + 5)(Ty + 2 guard + 5) and
 *                PF = (Tx + 2 guard + 4)(Ty + 2 guard + 4) are padded up to
 *                8 mod 16 and 8 mod 32 words (150,720 B for 8x8x8, guard 1).
 *   threads      threads per tile workgroup (256, 512 or 1024; 0 = 512).
 *   interleave   order of the particles inside a tile after a sort.
 *                0 (default): level order -- level r holds the (r+1)-th
 *                particle of every cell that has one, cells in key order,
 *                levels one after another, so a wavefront's lanes hold
 *                different cells at any density.  D >= 1: each full block
 *                of 64 D cell-sorted particles is stored D x 64 transposed
 *                (lanes D apart in cell order; 1 = plain cell order). */
typedef struct {
    int32_t n[3];
    int32_t solver;
    double d[3];
    double dt;
    int32_t pd_variant;
    int32_t bc_x;
    int32_t jpost;
    int32_t tile[3];
    int32_t sort_interval;
    int32_t guard;
    int32_t threads;
    int32_t interleave;
} pic_grid_desc;

/* Caller-owned FP32 device arrays, each n[0]*n[1]*n[2] values (layout above). */
typedef struct {
    float *E[3];
    float *B[3];
    float *J[3];
} pic_field_bufs;

/* Caller-owned particle arrays of one species (device memory, SoA, `capacity`
 * entries each).  q, m in units of e, m_e. */
typedef struct {
    double q, m;
    int64_t capacity;
    int32_t *cell;
    float *off[3];
    float *u[3];
    float *w;
    int32_t *id;
} pic_species_bufs;

/* FP64 diagnostics (pic_reduce). */
typedef struct {
    double charge;      /* sum q w dV over live particles */
    double e_field;     /* 1/2 sum (E^2 + B^2) dV */
    double e_kin;       /* sum m w (gamma - 1) dV */
    double max_abs_J;   /* max |J| over the three components */
    int64_t n_particles;/* live particles over all species */
    int64_t step;       /* completed steps */
} pic_diag;

/* Laser pulse launched in +x through the plane x = src_x dx (Section 3.1: a
 * linearly polarised Gaussian pulse, polarised along y, entering from the
 * plasma border).  Built from the vector potential
 *   A_y(t) = a0 env(t) cos(omega0 (t - t_peak)),
 *   env(t) = exp(-2 ln2 (t - t_peak)^2 / fwhm^2)   (intensity FWHM = fwhm),
 * with E_y = -dA_y/dt (no DC part even for sub-cycle pulses) and transverse
 * profile exp(-((y-yc)^2 + (z-zc)^2) / waist^2).  The incident wave
 * E_y = B_z = e(t - (x - x_src)) f(y,z) enters through total-field /
 * scattered-field corrections on the B_z plane behind and the E_y plane on
 * the source, applied while t <= t_end and the window has not moved.
 * Units: a0 in m_e c/e, omega0 in w_pe, lengths c/w_pe, times 1/w_pe. */
typedef struct {
    double a0, omega0, waist, fwhm, t_peak, t_end, yc, zc;
    int32_t src_x;
    int32_t pad_;
} pic_laser_desc;

/* Cold electron plasma of a species, loaded on a regular sub-cell lattice of
 * ppc[0] x ppc[1] x ppc[2] particles per cell at offsets (k + 1/2)/ppc_d.
 * Density along the lab-frame x (in cells): 0 before x_start, rising
 * linearly over `ramp` cells, then n_plateau (in n0); each particle's weight
 * is n(x_lab)/ppc at its own lab position; none is loaded where n = 0.
 * Particle tag: ((X ny + j) nz + k) ppc + s (mod 2^31), X the lab cell,
 * (j, k) the transverse cell, s the lattice slot. */
typedef struct {
    double x_start, ramp, n_plateau;
    int32_t ppc[3];
    int32_t pad_;
} pic_plasma_desc;

/* Device time of the phases of pic_step, measured with HIP events on the
 * context's stream between pic_profile_enable and pic_profile_read
 * (milliseconds, summed over steps and species). */
typedef struct {
    double sort_ms;      /* cell sorts */
    double tile_ms;      /* fused tiled gather + push + deposit launches */
    double loose_ms;     /* rest pass: particles beyond their tile's guard or appended since the last sort */
    double jpost_ms;     /* current read-out and post-processing */
    double field_ms;     /* B half step, E step, B half step (+ laser source) */
    double window_ms;    /* window motion and plasma injection */
    int64_t steps, sorts, tile_launches;
} pic_profile;

typedef struct pic_ctx pic_ctx;

/* Bytes of device workspace pic_init_grid needs for this grid and a total
 * particle capacity (summed over species) of max_particles.  Pure host. */
size_t pic_workspace_bytes(const pic_grid_desc *desc, int64_t max_particles);

/* Validate a descriptor without touching the GPU.  On error writes a message
 * into msg (host, msg_len bytes, may be NULL).  Pure host. */
pic_status pic_validate_grid(const pic_grid_desc *desc, char *msg, size_t msg_len);

/* Create a context.  desc, fields: host structs, copied.  workspace: device
 * buffer of at least pic_workspace_bytes(desc, max_particles) bytes, 256-byte
 * aligned, owned by the caller and kept alive until pic_destroy.  stream:
 * hipStream_t of the caller (NULL = default stream).  On success *out holds
 * the new context; on failure *out is NULL.  Fields are not modified. */
pic_status pic_init_grid(pic_ctx **out, const pic_grid_desc *desc, const pic_field_bufs *fields,
                         void *workspace, size_t workspace_bytes, int64_t max_particles, void *stream);

/* Register a species.  bufs: host struct, copied; the arrays must already
 * hold n_particles valid particles (0 <= n_particles <= capacity), each with
 * cell in [0, ncells) and off in [0, 1).  *species_out (host) receives the
 * species index.  Asynchronous. */
pic_status pic_init_species(pic_ctx *ctx, const pic_species_bufs *bufs, int64_t n_particles,
                            int32_t *species_out);

/* Field gather + Boris push + move for one species: x^n, u^{n-1/2} ->
 * x^{n+1}, u^{n+1/2}, using E^n, B^n.  This is the particle half of the PIC
 * cycle of Section 1 (particles in continuous phase space driven by the
 * grid fields); the paper's advance of the macroparticles is the cost it
 * names as dominant (Section 1).  The interpolation is the third-order
 * (cubic) B-spline of the macroparticle shapes (Sections 1 and 3.1) taken
 * at each field component's own staggered position.  The paper does not
 * name its pusher: this library uses the relativistic Boris rotation.
 * Keeps x^n in the workspace for pic_deposit.  Asynchronous. */
pic_status pic_gather_push(pic_ctx *ctx, int32_t species);

/* The current J of eq. 2.1, "deposited from particle motion" (Section 2),
 * for the species' motion x^n -> x^{n+1} of the last pic_gather_push, with
 * the cubic shapes of Sections 1 and 3.1.  The paper does not name the
 * deposition scheme: this library uses Esirkepov's charge-conserving
 * decomposition, so the discrete continuity equation holds exactly for the
 * charge the same shapes deposit.  Contributions are summed in an exact
 * int64 fixed-point accumulator (2^-40 units; independent of order), then J
 * (FP32) is set to the accumulated current of all species deposited since
 * the last field step.  Asynchronous. */
pic_status pic_deposit(pic_ctx *ctx, int32_t species);

/* J post-processing (desc.jpost), then B^{n+1/2} = B^n - dt/2 curl'E^n,
 * E^{n+1} = E^n + dt (curl B^{n+1/2} - J), B^{n+1} = B^{n+1/2} - dt/2 curl'E^{n+1}
 * (Section 2, eq. 2.1), then clears the current accumulator.  After a
 * filter, J holds the filtered current.  Asynchronous. */
pic_status pic_field_step(pic_ctx *ctx);

/* nsteps full production steps of the PIC cycle of Section 1 (fields on
 * the grid advanced by eq. 2.1 of Section 2, particles advanced in
 * continuous phase space) with the moving window of Section 1: periodic
 * cell sort, fused tiled gather+push+deposit of every species, J
 * post-processing, field update and window motion.  Equal to
 * pic_gather_push + pic_deposit (all species) + pic_field_step per step,
 * bit for bit.  Asynchronous. */
pic_status pic_step(pic_ctx *ctx, int32_t nsteps);

/* Counting sort of one species by tile and cell; drops removed particles.
 * Not part of the paper's method: a data layout of this library (particles
 * of one tile are contiguous so the fused step can stage the tile's fields
 * and current in on-chip memory); it changes no result.
 * Tiles of 8 x 2m x 4k cells are keyed in 8x2x4-cell bricks (x fastest,
 * then z, then y inside a brick), other tiles in x-fastest cell order; the
 * particles of a tile are then stored in the order the tiling's interleave
 * selects (level order, or a block transpose).  The
 * species' data may move to the workspace copy (see pic_species_view).
 * Asynchronous. */
pic_status pic_sort(pic_ctx *ctx, int32_t species);

/* Current device arrays and live count of a species (host struct out).
 * Synchronises the stream and reports device-side errors. */
pic_status pic_species_view(pic_ctx *ctx, int32_t species, pic_species_bufs *out, int64_t *n_live);

/* Continuity check of the last gather_push/deposit pair (the charge
 * conservation that the current of eq. 2.1 must obey), FP64 on the device:
 * max over nodes of |(rho^{n+1} - rho^n) dx/dt + sum_d (dx/d_d)(J_d - J_d[-e_d])|
 * with rho deposited in FP64 from the stored FP32 positions and J the FP32
 * current in the J planes.  When those hold the post-processed current
 * (after the field step or pic_current_filter of a grid with jpost binomial
 * or the denoiser, whose output B(J + sigma curl y) has the divergence of
 * B J), rho passes through the same binomial stencil B first: the
 * post-processed current conserves the filtered charge.  Right after
 * pic_deposit the planes hold the raw current and rho is used as is.
 * *resid and *max_abs_j are host outputs.  Synchronises. */
pic_status pic_continuity(pic_ctx *ctx, int32_t species, double *resid, double *max_abs_j);

/* pic_continuity without the workspace: for callers that cannot allocate
 * device memory themselves (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * synchronisation as pic_continuity, but its scratch (the FP64 charge
 * density and the reduction words) is a fixed device array of the library,
 * 16 MiB + 256 B per GPU, held until the process ends; it allocates
 * nothing and writes nothing to the workspace's density buffer.  Grids of
 * more than 2^21 cells are refused (PIC_EINVAL).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other threads or
 * streams) race.  The array is cleared by a kernel at each call. */
pic_status pic_continuity_noalloc(pic_ctx *ctx, int32_t species, double *resid, double *max_abs_j);

/* FP64 diagnostics (host output): total charge, field energy, kinetic
 * energy, max |J| and the live particle count (pic_diag).  Section 3 names
 * grid heating among the numerical artefacts a predictive code must not
 * introduce; the field and kinetic energy sums are what watching for it
 * takes.  Synchronises; reports device errors. */
pic_status pic_reduce(pic_ctx *ctx, pic_diag *host_out);

/* Wait for queued work; report device-side errors. */
pic_status pic_sync(pic_ctx *ctx);

/* Laser source (host struct, copied; NULL removes it).  src_x must lie in
 * [1, n[0] - 1); in moving-window mode the window must not start moving
 * before t_end (checked by pic_set_window and here). */
pic_status pic_set_laser(pic_ctx *ctx, const pic_laser_desc *laser);

/* Plasma profile of a species (host struct, copied), used by
 * pic_inject_plasma and by the moving window's injection of each newly
 * covered slab. */
pic_status pic_set_plasma(pic_ctx *ctx, int32_t species, const pic_plasma_desc *plasma);

/* Append the species' cold plasma of window cells x in [x_begin, x_end) (all
 * y, z) at the current window position.  Fails with PIC_ENOMEM if the
 * species capacity could be exceeded (host-side bound); particles land
 * outside the tile ranges until the next sort.  Asynchronous. */
pic_status pic_inject_plasma(pic_ctx *ctx, int32_t species, int32_t x_begin, int32_t x_end);

/* Moving window (desc.bc_x = PIC_BC_MOVING_WINDOW): after every step whose
 * index + 1 >= start_step, the window advances one cell in +x at c (c dt =
 * dx is required for this): the plane leaving at the back becomes the new
 * leading plane with zero fields, and each species with a plasma profile
 * gets the plasma of the newly covered cells loaded at window cell
 * n[0] - 4.  Particles outside window cells [3, n[0] - 4] are removed (their
 * shapes would reach across the window's ends). */
pic_status pic_set_window(pic_ctx *ctx, int64_t start_step);

/* Cells the window has moved and the storage x index of window cell 0
 * (host outputs). */
pic_status pic_window_state(pic_ctx *ctx, int64_t *shift, int32_t *origin);

/* ---- Transverse absorbing layer --------------------------------------------
 *
 * Section 3.1 surrounds its Cartesian box transversely with a 16-layer
 * perfectly matched layer.  With a layer set, y and z are no longer
 * periodic: the `layers` outermost cells at each y and z edge form the
 * layer, fields beyond the outer faces are zero, and every transverse
 * derivative D of the curls inside the layer is stretched in the
 * convolutional form (D -> D + psi, psi <- b psi + (b - 1) D,
 * b = exp(-sigma dt), no frequency shift, unit kappa).  Grading: at
 * position p in cells (integer for nodes, half-integer for face centres)
 * along an axis of n cells, depth = max((L - 1 - p) / L, (p - (n - L)) / L)
 * clipped to [0, 1] and sigma = sigma_max depth^grade (zero on nodes
 * L - 1 .. n - L).  The B arrays advance once per step, at the first B half
 * step, as the leapfrog recursion of B between half-integer times.
 * Particles whose transverse cell lies in the layer are removed at the
 * start of the next step (like the window's kill zones; pic_reduce and the
 * diagnostics no longer count them).  The auxiliary arrays move with the
 * window and are part of the checkpoint blob. */
typedef struct {
    int32_t layers;         /* L: cells per edge, 8 <= L, 2 L + 1 <= n[1], n[2]; 0 removes the layer */
    int32_t pad_;
    double sigma_max[2];    /* y, z in w_pe (<= 0: 0.8 (grade + 1) / d, the usual optimum) */
    double grade;           /* profile exponent (<= 0: 3) */
} pic_pml_desc;

/* Device bytes the layer's arrays need (pure host; 0 for an invalid descriptor). */
size_t pic_pml_bytes(const pic_grid_desc *desc, const pic_pml_desc *pml);

/* Set (or with layers = 0 remove) the layer.  buffer: caller-owned device
 * memory of at least pic_pml_bytes, 256-byte aligned, kept until the
 * context is destroyed or the layer removed; zeroed here (the layer starts
 * empty).  Not with the batched launcher (pic_batch_create rejects such a
 * context).  Synchronises. */
pic_status pic_set_pml(pic_ctx *ctx, const pic_pml_desc *pml, void *buffer, size_t bytes);

/* ---- Run diagnostics -----------------------------------------------------
 *
 * The quantities Section 3.2 reports for its runs, computed on the device in
 * FP64 from the live state (synchronising calls; host outputs).  Positions
 * are window coordinates (x from the window's trailing face); particles in
 * the window's removal margins count as gone, as in pic_reduce.
 */

/* A field component (comp 0..5 = E_x, E_y, E_z, B_x, B_y, B_z) along x at
 * the transverse point (yc, zc): host_line[i], i < n[0], is the value at
 * window cell i of the component's staggered grid, bilinear in y and z
 * between the four nearest nodes (periodic y, z).  With comp 0 on the laser
 * axis this is the on-axis longitudinal field of Section 3.2, Fig. 1(a). */
pic_status pic_axis_line(pic_ctx *ctx, int32_t comp, double yc, double zc, double *host_line);

/* Length of the accelerating phase on the axis (yc, zc): the region inside
 * the bubble where E_x < 0 (Section 3.2, Fig. 1(a)).  Going backward from
 * the last E_x sample at or behind x_from (window coordinates, typically
 * the laser centroid), samples with E_x >= 0 (the front of the bubble) are
 * skipped; the accelerating phase is the run of negative samples that
 * follows, its ends at the zero crossings interpolated linearly between
 * samples (a run reaching past x_from ends there).  0 if there is none. */
pic_status pic_accelerating_length(pic_ctx *ctx, double yc, double zc, double x_from, double *length);

/* Charge spectrum of a species: the charge |q| w dV of its live particles
 * binned by kinetic energy gamma - 1 (quantity 0, in m_e c^2) or by the
 * longitudinal momentum u_x (quantity 1, in m_e c) over [lo, hi) in nbins
 * equal bins (1..2048); particles outside the range are not counted
 * (Section 3.2, Figs. 3-4; Section 3.3, momentum spectra).  host_charge:
 * nbins doubles; host_count (may be NULL): nbins particle counts. */
pic_status pic_spectrum(pic_ctx *ctx, int32_t species, int32_t quantity, double lo, double hi, int32_t nbins,
                        double *host_charge, int64_t *host_count);

/* Beam of the particles with u_x > ux_min: its charge, count, mean u_x and
 * normalised transverse emittances in y and z (Section 3.2, Table 1):
 * eps_N,i = [(<p_i^2> - <p_i>^2)(<r_i^2> - <r_i>^2) - (<p_i r_i> - <r_i><p_i>)^2]^(1/2)
 * with p in m_e c and r in c/w_pe (so eps in c/w_pe), averages weighted by
 * charge; also the centroid and spreads of r and p. */
typedef struct {
    double charge;
    int64_t count;
    double mean_ux;
    double eps_ny, eps_nz;
    double mean_r[2];   /* <y>, <z> */
    double rms_r[2];    /* spread of y, z */
    double rms_p[2];    /* spread of u_y, u_z */
} pic_beam_diag;

pic_status pic_beam_moments(pic_ctx *ctx, int32_t species, double ux_min, pic_beam_diag *out);

/* The particles with u_x > ux_min, for the collection phase space of
 * Section 3.2, Fig. 1(b), (c): their tags (from which the plasma loading
 * gives the initial position), window x and u_x, in no particular order.
 * Up to cap of them are written to host_id, host_x, host_ux; *n_selected
 * receives how many qualify.  Uses the species' spare particle arrays as
 * staging (free between steps). */
pic_status pic_select_particles(pic_ctx *ctx, int32_t species, double ux_min, int64_t cap, int32_t *host_id,
                                double *host_x, float *host_ux, int64_t *n_selected);

/* Moments of the electromagnetic energy density e = (E^2 + B^2)/2 along x:
 * host_out[0] = sum e dV, [1] = sum e x dV, [2] = sum e x^2 dV, each
 * component at its own staggered x position in window coordinates.
 * transverse_only != 0 uses E_y, E_z, B_y, B_z only (a pulse travelling
 * along x).  [1]/[0] is the laser centroid, whose motion gives the pulse's
 * group velocity (Section 3.3). */
pic_status pic_field_moments(pic_ctx *ctx, int32_t transverse_only, double *host_out);

/* ---- Checkpoint / resume ---------------------------------------------------
 *
 * A long laser-wakefield run (the paper's runs take 10^5 CPU-hours,
 * Section 3.1) is resumed from a host copy of its state.  The blob holds the
 * fields E, B, J, every species' particles (cell, off, u, w, id of the live
 * and not yet dropped entries), the step counter, the window's shift and
 * origin (which fix where the next plasma slab is loaded and whether the
 * laser source is active).  Configuration is not in the blob: a resumed run
 * is a context made with the same descriptor, the same species (capacities
 * at least the stored counts) and the same pic_set_laser / pic_set_plasma /
 * pic_set_window / pic_denoiser_set calls.  A resumed run reaches the same
 * fields and particles (by id) bit for bit as the uninterrupted one: the
 * current is summed in an order-independent fixed-point accumulator and
 * the cell sort changes no result.
 * Layout (host byte order): a header, then E[3], B[3], J[3] as
 * n[0]*n[1]*n[2] floats each, with a transverse absorbing layer its
 * auxiliary arrays (pic_pml_bytes minus the coefficient table), then for
 * each species its count entries of cell, off[0..2], u[0..2], w, id (4
 * bytes per value, array by array). */

/* Bytes pic_copy_out needs for the current state (host output).
 * Synchronises the stream and reports device errors. */
pic_status pic_checkpoint_bytes(pic_ctx *ctx, size_t *bytes);

/* Copy the state into host_blob (host memory of `bytes` bytes; PIC_ENOMEM
 * if too small).  PIC_ESTATE inside a split-path step (pic_gather_push
 * without the closing pic_field_step).  Synchronises. */
pic_status pic_copy_out(pic_ctx *ctx, void *host_blob, size_t bytes);

/* Restore a state written by pic_copy_out into a context with the same grid
 * (n, d, dt, solver, x boundary, absorbing layer thickness) and species count (PIC_EINVAL otherwise;
 * PIC_ENOMEM when a species' capacity is below its stored count).  The
 * caller's species arrays receive the particles; every species is re-sorted
 * at its next pic_step.  Synchronises. */
pic_status pic_copy_in(pic_ctx *ctx, const void *host_blob, size_t bytes);

/* Change the fused step's tiling on a live context (same meaning and
 * defaults as the pic_grid_desc fields; the LDS footprint must fit).  Every
 * species is re-sorted at its next pic_step.  Results do not depend on the
 * tiling (bit for bit).  Used by the autotuner. */
typedef struct {
    int32_t tile[3];
    int32_t guard;
    int32_t threads;
    int32_t interleave;
    int32_t sort_interval;
} pic_tiling;

pic_status pic_set_tiling(pic_ctx *ctx, const pic_tiling *tiling);

/* Start (enable != 0) or stop timing the phases of pic_step; starting
 * clears the accumulated times.  Creates HIP events on first use (host
 * runtime objects, no device memory). */
pic_status pic_profile_enable(pic_ctx *ctx, int32_t enable);

/* Accumulated phase times since pic_profile_enable (host output).
 * Synchronises the stream. */
pic_status pic_profile_read(pic_ctx *ctx, pic_profile *out);

/* Learned current denoiser (desc.jpost = PIC_JPOST_DENOISER).  Not part of
 * the paper: the paper fights particle noise in the current with cubic
 * shapes and many particles per cell (Sections 1, 3.1); this network is a
 * learned replacement for the binomial filter at few particles per cell.
 *   x  = bf16(J_d / scale_d)
 *   a1 = bf16(relu(conv(x,  W1) + b1)),  a2 = bf16(relu(conv(a1, W2) + b2))
 *   y  = conv(a2, W3) + b3
 *   J <- B(J + sigma curl(y)),   sigma = dx (scale_x + scale_y + scale_z) / 3
 * B is the binomial filter of PIC_JPOST_BINOMIAL and curl the
 * backward-difference curl of the E update, whose discrete divergence is
 * zero: the denoised current obeys the same discrete continuity equation as
 * the binomially filtered one (periodic axes), carries no grid-scale
 * (Nyquist) modes, and zero W3, b3 give exactly the filter.
 * conv: 3x3x3 cross-correlation, output size = input size; y and z
 * periodic, x periodic or, in a moving window, zero beyond the window's
 * ends.  Weights and activations bf16 (rounded to nearest even), FP32
 * accumulation and biases, on the matrix cores.
 * weights (host, FP32, copied and rounded to bf16): W1 [32][3][3][3][3],
 * then W2 [32][32][3][3][3], then W3 [3][32][3][3][3], each indexed
 * [out][in][z][y][x] with tap (z, y, x) = offsets (-1, 0, +1) + 1.
 * biases (host, FP32): b1[32], b2[32], b3[3].  scale (host): 3 values > 0.
 * Synchronises the stream. */
pic_status pic_denoiser_set(pic_ctx *ctx, const float *weights, const float *biases, const float *scale);

/* Apply the grid's current post-processing (desc.jpost) to J in place.
 * Asynchronous. */
pic_status pic_current_filter(pic_ctx *ctx);

/* Text of the sticky error (never NULL). */
const char *pic_last_error(const pic_ctx *ctx);

/* Release the context (host memory only; caller buffers are untouched). */
void pic_destroy(pic_ctx *ctx);

/* ---- Batched launcher --------------------------------------------------
 *
 * A batch advances many independent simulations (members: contexts made
 * with pic_init_grid / pic_init_species / pic_set_*) in lockstep with one
 * kernel launch per phase for all of them: the fused tile step's work list
 * is the concatenation of every member's tiles, and each cell, plane or
 * particle kernel indexes members by its grid's second dimension.  A member
 * reaches exactly (bit for bit) the state that its own pic_step would reach;
 * sort, window, laser and injection schedules stay per member.  This serves
 * parameter scans, the optimisation of accelerator parameters through many
 * simulations that Sections 1 and 3.3 point to: many uneven laser-wakefield
 * setups, none large enough alone to fill the GPU.  The batching itself is
 * this library's design, not the paper's.
 *
 * Per step the host writes a table of member descriptors into a slot of the
 * batch workspace (a ring of slots, so no step waits for the previous one)
 * through a small pinned host staging ring that the batch allocates with
 * hipHostMalloc and frees in pic_batch_destroy.
 */
typedef struct pic_batch pic_batch;

/* Device workspace a batch of n members needs (0 if n < 1). */
size_t pic_batch_workspace_bytes(int32_t n_members);

/* members: host array of n context pointers (distinct, each with the same
 * number of species >= 1, all created on `stream`).  The contexts stay owned
 * by the caller and must outlive the batch; between batch calls they may be
 * used directly (pic_reduce, pic_species_view, ...) on the same stream.
 * workspace: device buffer of pic_batch_workspace_bytes(n), 256-byte aligned,
 * owned by the caller.  The tile step runs with the first member's threads
 * per tile.  Synchronises the stream once. */
pic_status pic_batch_create(pic_batch **out, pic_ctx *const *members, int32_t n, void *workspace,
                            size_t workspace_bytes, void *stream);

/* nsteps production steps of every member (each equal to pic_step(member, 1)
 * per step).  Asynchronous, except for a host wait when the staging ring is
 * full or a member's plasma injection needs an exact particle count. */
pic_status pic_batch_step(pic_batch *batch, int32_t nsteps);

/* Wait for queued work; report the first member's device-side error. */
pic_status pic_batch_sync(pic_batch *batch);

/* Phase timing of pic_batch_step, as pic_profile_enable / pic_profile_read
 * (tile_launches counts batched tile launches). */
pic_status pic_batch_profile_enable(pic_batch *batch, int32_t enable);
pic_status pic_batch_profile_read(pic_batch *batch, pic_profile *out);

/* Text of the batch's sticky error (never NULL). */
const char *pic_batch_last_error(const pic_batch *batch);

/* Release the batch (its pinned staging ring and events; members and
 * buffers are untouched).  Synchronises the stream. */
void pic_batch_destroy(pic_batch *batch);

/* ---- Denoiser training --------------------------------------------------
 *
 * Trains the pic_denoiser_set network on pairs of currents: an input J
 * deposited by few particles per cell and a target J_target deposited by
 * many (the same plasma), on crops of n[0] x n[1] x n[2] cells with zero
 * beyond the crop's faces.  Loss: mean over cells and the 3 components of
 * ((J' - J_target) / scale)^2 with J' the network's output current.
 * Forward and backward run on the bf16 matrix
 * cores with FP32 accumulation; parameters are FP32 master weights updated
 * by Adam (beta1 0.9, beta2 0.999, eps 1e-8), rounded to bf16 for every
 * convolution.  Weight and bias layouts are those of pic_denoiser_set.
 */
typedef struct pic_dn_trainer pic_dn_trainer;

/* Device workspace for crops of crop[3] cells (0 when invalid). */
size_t pic_dn_trainer_workspace_bytes(const int32_t crop[3]);

/* cell (host): the crops' cell sizes dx, dy, dz.  workspace: caller-owned
 * device buffer, 256-byte aligned, kept until destroy.  stream: the
 * caller's hipStream_t. */
pic_status pic_dn_trainer_create(pic_dn_trainer **out, const int32_t crop[3], const double cell[3], void *workspace,
                                 size_t workspace_bytes, void *stream);

/* Load parameters (host, FP32) and scales; resets the optimiser state.
 * Synchronises. */
pic_status pic_dn_trainer_set_params(pic_dn_trainer *tr, const float *weights, const float *biases,
                                     const float *scale);

/* Current FP32 master parameters (host outputs).  Synchronises. */
pic_status pic_dn_trainer_get_params(pic_dn_trainer *tr, float *weights, float *biases);

/* One Adam step on one crop.  input[3], target[3]: device FP32 component
 * arrays of n[0]*n[1]*n[2] values (x fastest).  *loss (host, may be NULL)
 * receives the loss before the update; asynchronous when loss is NULL. */
pic_status pic_dn_trainer_step(pic_dn_trainer *tr, float *const input[3], float *const target[3], float lr,
                               double *loss);

/* One Adam step on the mean gradient of a mini-batch of n crops.
 * inputs, targets: host arrays of 3 n device pointers (crop i's components
 * at 3 i .. 3 i + 2).  *loss (host, may be NULL): mean loss of the batch
 * before the update. */
pic_status pic_dn_trainer_step_batch(pic_dn_trainer *tr, int32_t n, float *const *inputs, float *const *targets,
                                     float lr, double *loss);

/* Mean loss over n crops (same array convention), no update.  Synchronises. */
pic_status pic_dn_trainer_eval(pic_dn_trainer *tr, int32_t n, float *const *inputs, float *const *targets,
                               double *loss);

/* Loss and gradients without an update (host outputs, pic_denoiser_set
 * layouts).  Synchronises. */
pic_status pic_dn_trainer_grad(pic_dn_trainer *tr, float *const input[3], float *const target[3], double *loss,
                               float *grad_weights, float *grad_biases);

/* freeze != 0: later updates leave the biases at their current values
 * (with zero biases the network maps J = 0 to no correction and scales
 * with its input: net(a J) = a net(J) for a > 0). */
pic_status pic_dn_trainer_freeze_biases(pic_dn_trainer *tr, int32_t freeze);

const char *pic_dn_trainer_last_error(const pic_dn_trainer *tr);
void pic_dn_trainer_destroy(pic_dn_trainer *tr);

#ifdef __cplusplus
}
#endif

#endif /* PIC355_H */
