/*
 * FP64 reference implementation of the explicit particle-in-cell cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  The product
 * path (the HIP library) never links, calls or includes anything from here,
 * and this file includes nothing from the product path.
 *
 * It is deliberately plain and slow: one particle at a time, one node at a
 * time, in double precision, in the order the method states its steps:
 *
 *   field gather (cubic B-spline at each component's staggered position)
 *   -> relativistic Boris push -> move -> charge-conserving current deposit
 *   (Esirkepov's density decomposition, cubic shapes) -> optional binomial
 *   current filter -> FDTD update B(n+1/2), E(n+1), B(n+1).
 *
 * The field update is the paper's eq. (2.1): D_t B = -curl' E,
 * D_t E = c^2 curl B - J/eps0 (normalised: c = eps0 = 1), where curl' takes
 * D_i S_i in place of D_i (Section 2), and S_x is the 3x3 transverse stencil
 * of Section 2 (centre alpha_x, +-y neighbours beta_y, +-z neighbours beta_z,
 * corners gamma_yz; S_y, S_z by cyclic permutation).  With alpha = 1 and
 * beta = gamma = 0 every S_i is the identity and the update is the standard
 * Yee scheme (Section 1).  The PIC cycle itself is the one the introduction
 * describes (fields on a grid, particles in continuous phase space).
 *
 * Layout: field component arrays of nx*ny*nz doubles, x fastest, index
 * (i,j,k) -> i + nx*(j + ny*k).  Yee staggering: E_x(i+1/2,j,k),
 * E_y(i,j+1/2,k), E_z(i,j,k+1/2), B_x(i,j+1/2,k+1/2), B_y(i+1/2,j,k+1/2),
 * B_z(i+1/2,j+1/2,k); J like E; rho on nodes (i,j,k).  Array index (i,j,k)
 * holds the value at the staggered point whose integer parts are (i,j,k).
 * Particles: absolute positions x[3][np] in c/w_p, momenta u = gamma v/c,
 * density weights w (n/ppc).  y and z are periodic; x is periodic or, for a
 * moving window, bounded by zero-valued ghost fields.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n[3];     /* cells */
    double d[3];      /* cell sizes */
    double dt;        /* time step */
    int32_t xbc;      /* 0: periodic in x; 1: zero ghost beyond both x edges */
    int32_t yzbc;     /* bit 0: zero beyond the y edges, bit 1: beyond the z edges (else periodic) */
    double alpha[3];  /* centre weights of S_x, S_y, S_z */
    double beta[3];   /* beta_x, beta_y, beta_z */
    double gam[3];    /* gamma_yz, gamma_zx, gamma_xy */
} ora_grid;

enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENONFINITE = -5 };

/* ------------------------------------------------------------------ */
/* grid helpers                                                        */

static int64_t wrap(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t ncell(const ora_grid *g) { return g->n[0] * g->n[1] * g->n[2]; }

/* Value of a field component at integer index (i,j,k) with the boundary rule:
 * y, z periodic; x periodic or zero outside [0, nx). */
static double fld(const ora_grid *g, const double *F, int64_t i, int64_t j, int64_t k) {
    if (g->xbc == 1) {
        if (i < 0 || i >= g->n[0]) return 0.0;
    } else {
        i = wrap(i, g->n[0]);
    }
    if ((g->yzbc & 1) && (j < 0 || j >= g->n[1])) return 0.0;
    if ((g->yzbc & 2) && (k < 0 || k >= g->n[2])) return 0.0;
    j = wrap(j, g->n[1]);
    k = wrap(k, g->n[2]);
    return F[i + g->n[0] * (j + g->n[1] * k)];
}

/* Flat index of (i,j,k) or -1 when x falls outside a bounded window. */
static int64_t node(const ora_grid *g, int64_t i, int64_t j, int64_t k) {
    if (g->xbc == 1) {
        if (i < 0 || i >= g->n[0]) return -1;
    } else {
        i = wrap(i, g->n[0]);
    }
    if ((g->yzbc & 1) && (j < 0 || j >= g->n[1])) return -1;
    if ((g->yzbc & 2) && (k < 0 || k >= g->n[2])) return -1;
    j = wrap(j, g->n[1]);
    k = wrap(k, g->n[2]);
    return i + g->n[0] * (j + g->n[1] * k);
}

/* ------------------------------------------------------------------ */
/* shape                                                               */

/* Cubic (third-order) B-spline of support 4 cells, the macroparticle shape
 * named in Sections 1 and 3.1: S(xi) = 2/3 - xi^2 + |xi|^3/2 for |xi| < 1,
 * (2-|xi|)^3/6 for 1 <= |xi| < 2, 0 beyond. */
double ora_bspline3(double xi) {
    double a = fabs(xi);
    if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
    if (a < 2.0) {
        double t = 2.0 - a;
        return t * t * t / 6.0;
    }
    return 0.0;
}

/* Staggering of the six field components: offset (0 or 1/2 cell) per axis. */
static const double STAG_E[3][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
static const double STAG_B[3][3] = {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

/* Interpolate component array F (staggered by sh[3]) at absolute position x. */
static double gather1(const ora_grid *g, const double *F, const double sh[3], const double x[3]) {
    int64_t base[3];
    double wgt[3][4];
    for (int a = 0; a < 3; ++a) {
        double s = x[a] / g->d[a] - sh[a];
        int64_t i = (int64_t)floor(s);
        base[a] = i - 1;
        for (int m = 0; m < 4; ++m) wgt[a][m] = ora_bspline3((double)(base[a] + m) - s);
    }
    double acc = 0.0;
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a)
                acc += fld(g, F, base[0] + a, base[1] + b, base[2] + c) * wgt[0][a] * wgt[1][b] * wgt[2][c];
    return acc;
}

/* Field gather at one position: each component with a cubic spline at its
 * own staggered grid (momentum-conserving interpolation). */
void ora_gather(const ora_grid *g, const double *E, const double *B, const double x[3],
                double Ep[3], double Bp[3]) {
    int64_t nc = ncell(g);
    for (int c = 0; c < 3; ++c) {
        Ep[c] = gather1(g, E + c * nc, STAG_E[c], x);
        Bp[c] = gather1(g, B + c * nc, STAG_B[c], x);
    }
}

/* Relativistic Boris rotation, u = gamma v / c, normalised units:
 * h = q dt / (2 m); u- = u + h E; t = h B / gamma(u-); s = 2t/(1+t^2);
 * u' = u- + u- x t; u+ = u- + u' x s; u_new = u+ + h E. */
void ora_boris(double u[3], const double Ep[3], const double Bp[3], double qm, double dt) {
    double h = 0.5 * qm * dt;
    double um[3] = {u[0] + h * Ep[0], u[1] + h * Ep[1], u[2] + h * Ep[2]};
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {h * Bp[0] / gm, h * Bp[1] / gm, h * Bp[2] / gm};
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
    double up[3] = {um[0] + um[1] * t[2] - um[2] * t[1],
                    um[1] + um[2] * t[0] - um[0] * t[2],
                    um[2] + um[0] * t[1] - um[1] * t[0]};
    double upl[3] = {um[0] + up[1] * s[2] - up[2] * s[1],
                     um[1] + up[2] * s[0] - up[0] * s[2],
                     um[2] + up[0] * s[1] - up[1] * s[0]};
    for (int a = 0; a < 3; ++a) u[a] = upl[a] + h * Ep[a];
}

/* Gather + Boris + move for every particle.  x is read at time n, u at n-1/2;
 * on return u is at n+1/2, x_new (unwrapped, x^n + dt u/gamma) at n+1 and x
 * holds x_new wrapped into the periodic box. */
int ora_push(const ora_grid *g, int64_t np, double *x, double *u, double *x_new,
             double q, double m, const double *E, const double *B) {
    int bad = 0;
    for (int64_t p = 0; p < np; ++p) {
        double xp[3] = {x[p], x[np + p], x[2 * np + p]};
        double up[3] = {u[p], u[np + p], u[2 * np + p]};
        double Ep[3], Bp[3];
        ora_gather(g, E, B, xp, Ep, Bp);
        ora_boris(up, Ep, Bp, q / m, g->dt);
        double gam = sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(up[a])) bad = 1;
            u[a * np + p] = up[a];
            double xn = xp[a] + g->dt * up[a] / gam;
            x_new[a * np + p] = xn;
            double L = g->n[a] * g->d[a];
            if (a == 0 && g->xbc == 1) {
                x[p] = xn;
            } else {
                x[a * np + p] = xn - L * floor(xn / L);
            }
        }
    }
    return bad ? ORA_ENONFINITE : ORA_OK;
}

/* ------------------------------------------------------------------ */
/* charge-conserving current deposit                                   */

/* Esirkepov's decomposition for one particle moving from x0 to x1 (x1 not
 * wrapped).  Per axis the union support is the 5 nodes base..base+4 with
 * base = min(floor(s0), floor(s1)) - 1, s = x/d.  With S0, S1 the cubic
 * weights of the old and new position and dS = S1 - S0:
 *   W^x_abc = dSx_a (S0y_b S0z_c + dSy_b S0z_c/2 + S0y_b dSz_c/2 + dSy_b dSz_c/3)
 * (and cyclically for y, z); the current is the running sum along its axis:
 *   J_x(base_x+a+1/2, base_y+b, base_z+c) += -q w (dx/dt) sum_{a'<=a} W^x_{a'bc}.
 * Summed over axes, W gives S1S1S1 - S0S0S0, so the discrete continuity
 * equation holds exactly. */
void ora_deposit_one(const ora_grid *g, const double x0[3], const double x1[3], double w, double q,
                     double *J) {
    int64_t nc = ncell(g);
    int64_t base[3];
    double S0[3][5], dS[3][5];
    for (int a = 0; a < 3; ++a) {
        double s0 = x0[a] / g->d[a], s1 = x1[a] / g->d[a];
        int64_t i0 = (int64_t)floor(s0), i1 = (int64_t)floor(s1);
        base[a] = (i0 < i1 ? i0 : i1) - 1;
        for (int m = 0; m < 5; ++m) {
            double node_pos = (double)(base[a] + m);
            S0[a][m] = ora_bspline3(node_pos - s0);
            dS[a][m] = ora_bspline3(node_pos - s1) - S0[a][m];
        }
    }
    for (int comp = 0; comp < 3; ++comp) {
        /* comp = direction of the current; (t1, t2) the two other axes */
        int t1 = (comp + 1) % 3, t2 = (comp + 2) % 3;
        double coef = -q * w * g->d[comp] / g->dt;
        for (int b = 0; b < 5; ++b)
            for (int c = 0; c < 5; ++c) {
                double trans = S0[t1][b] * S0[t2][c] + 0.5 * dS[t1][b] * S0[t2][c] +
                               0.5 * S0[t1][b] * dS[t2][c] + dS[t1][b] * dS[t2][c] / 3.0;
                double run = 0.0;
                for (int a = 0; a < 5; ++a) {
                    run += dS[comp][a] * trans;
                    int64_t idx[3];
                    idx[comp] = base[comp] + a;
                    idx[t1] = base[t1] + b;
                    idx[t2] = base[t2] + c;
                    int64_t f = node(g, idx[0], idx[1], idx[2]);
                    if (f >= 0) J[comp * nc + f] += coef * run;
                }
            }
    }
}

/* J += deposit of all particles moving x0 -> x1 (x1 unwrapped). */
void ora_deposit(const ora_grid *g, int64_t np, const double *x0, const double *x1, const double *w,
                 double q, double *J) {
    for (int64_t p = 0; p < np; ++p) {
        double a[3] = {x0[p], x0[np + p], x0[2 * np + p]};
        double b[3] = {x1[p], x1[np + p], x1[2 * np + p]};
        ora_deposit_one(g, a, b, w[p], q, J);
    }
}

/* Charge density on nodes: rho(i,j,k) += q w S S S (cubic shape at the node grid). */
void ora_rho(const ora_grid *g, int64_t np, const double *x, const double *w, double q, double *rho) {
    for (int64_t p = 0; p < np; ++p) {
        int64_t base[3];
        double wgt[3][4];
        for (int a = 0; a < 3; ++a) {
            double s = x[a * np + p] / g->d[a];
            int64_t i = (int64_t)floor(s);
            base[a] = i - 1;
            for (int m = 0; m < 4; ++m) wgt[a][m] = ora_bspline3((double)(base[a] + m) - s);
        }
        for (int c = 0; c < 4; ++c)
            for (int b = 0; b < 4; ++b)
                for (int a = 0; a < 4; ++a) {
                    int64_t f = node(g, base[0] + a, base[1] + b, base[2] + c);
                    if (f >= 0) rho[f] += q * w[p] * wgt[0][a] * wgt[1][b] * wgt[2][c];
                }
    }
}

/* Continuity residual on nodes: (rho1 - rho0) dx/dt + sum_d (dx/d_d)(J_d - J_d[-e_d]).
 * Writes it to res (may be NULL) and returns max |res|. */
double ora_continuity(const ora_grid *g, const double *rho0, const double *rho1, const double *J,
                      double *res) {
    int64_t nc = ncell(g);
    double mx = 0.0;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t f = i + g->n[0] * (j + g->n[1] * k);
                double r = (rho1[f] - rho0[f]) * g->d[0] / g->dt;
                r += (fld(g, J, i, j, k) - fld(g, J, i - 1, j, k));
                r += (g->d[0] / g->d[1]) * (fld(g, J + nc, i, j, k) - fld(g, J + nc, i, j - 1, k));
                r += (g->d[0] / g->d[2]) * (fld(g, J + 2 * nc, i, j, k) - fld(g, J + 2 * nc, i, j, k - 1));
                if (res) res[f] = r;
                if (fabs(r) > mx) mx = fabs(r);
            }
    return mx;
}

/* ------------------------------------------------------------------ */
/* field update                                                        */

/* Transverse smoothing S_d of component array F at (i,j,k), Section 2:
 * centre alpha_d, the two transverse axes t1 = d+1, t2 = d+2 (cyclic) with
 * neighbour weights beta_t1, beta_t2 and corner weight gamma_{t1 t2}. */
static double smooth(const ora_grid *g, const double *F, int d, int64_t i, int64_t j, int64_t k) {
    int64_t p[3] = {i, j, k};
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    double acc = g->alpha[d] * fld(g, F, i, j, k);
    for (int s = -1; s <= 1; s += 2) {
        int64_t q1[3] = {p[0], p[1], p[2]};
        q1[t1] += s;
        acc += g->beta[t1] * fld(g, F, q1[0], q1[1], q1[2]);
        int64_t q2[3] = {p[0], p[1], p[2]};
        q2[t2] += s;
        acc += g->beta[t2] * fld(g, F, q2[0], q2[1], q2[2]);
        for (int s2 = -1; s2 <= 1; s2 += 2) {
            int64_t qc[3] = {p[0], p[1], p[2]};
            qc[t1] += s;
            qc[t2] += s2;
            acc += g->gam[d] * fld(g, F, qc[0], qc[1], qc[2]);
        }
    }
    return acc;
}

/* Forward difference of S_d F along axis d at (i,j,k): (S_d F(p+e_d) - S_d F(p)) / d_d. */
static double dsmooth(const ora_grid *g, const double *F, int d, int64_t i, int64_t j, int64_t k) {
    int64_t q[3] = {i, j, k};
    q[d] += 1;
    return (smooth(g, F, d, q[0], q[1], q[2]) - smooth(g, F, d, i, j, k)) / g->d[d];
}

/* Backward difference of F along axis d at (i,j,k): (F(p) - F(p-e_d)) / d_d. */
static double dback(const ora_grid *g, const double *F, int d, int64_t i, int64_t j, int64_t k) {
    int64_t q[3] = {i, j, k};
    q[d] -= 1;
    return (fld(g, F, i, j, k) - fld(g, F, q[0], q[1], q[2])) / g->d[d];
}

/* B -= h curl' E  (B on faces, forward differences of the smoothed E). */
static void b_half(const ora_grid *g, const double *E, double *B, double h) {
    int64_t nc = ncell(g);
    double *tmp = (double *)malloc(sizeof(double) * 3 * nc);
    const double *Ex = E, *Ey = E + nc, *Ez = E + 2 * nc;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t f = i + g->n[0] * (j + g->n[1] * k);
                /* (curl' E)_x = D_y S_y E_z - D_z S_z E_y, and cyclic */
                tmp[f] = dsmooth(g, Ez, 1, i, j, k) - dsmooth(g, Ey, 2, i, j, k);
                tmp[nc + f] = dsmooth(g, Ex, 2, i, j, k) - dsmooth(g, Ez, 0, i, j, k);
                tmp[2 * nc + f] = dsmooth(g, Ey, 0, i, j, k) - dsmooth(g, Ex, 1, i, j, k);
            }
    for (int64_t f = 0; f < 3 * nc; ++f) B[f] -= h * tmp[f];
    free(tmp);
}

/* E += dt (curl B - J)  (E on edges, backward differences of B). */
static void e_full(const ora_grid *g, double *E, const double *B, const double *J) {
    int64_t nc = ncell(g);
    double *tmp = (double *)malloc(sizeof(double) * 3 * nc);
    const double *Bx = B, *By = B + nc, *Bz = B + 2 * nc;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t f = i + g->n[0] * (j + g->n[1] * k);
                tmp[f] = dback(g, Bz, 1, i, j, k) - dback(g, By, 2, i, j, k);
                tmp[nc + f] = dback(g, Bx, 2, i, j, k) - dback(g, Bz, 0, i, j, k);
                tmp[2 * nc + f] = dback(g, By, 0, i, j, k) - dback(g, Bx, 1, i, j, k);
            }
    for (int64_t f = 0; f < 3 * nc; ++f) E[f] += g->dt * (tmp[f] - (J ? J[f] : 0.0));
    free(tmp);
}

/* One field step: B^{n+1/2} = B^n - dt/2 curl'E^n; E^{n+1} = E^n + dt (curl B^{n+1/2} - J^{n+1/2});
 * B^{n+1} = B^{n+1/2} - dt/2 curl'E^{n+1}. */
void ora_field_step(const ora_grid *g, double *E, double *B, const double *J) {
    b_half(g, E, B, 0.5 * g->dt);
    e_full(g, E, B, J);
    b_half(g, E, B, 0.5 * g->dt);
}

/* Only the first half of the B update (used to check B at half steps). */
void ora_b_half(const ora_grid *g, const double *E, double *B, double h) { b_half(g, E, B, h); }

/* Discrete divergences: div E (on nodes) and div B (on cell centres). */
void ora_div_e(const ora_grid *g, const double *E, double *out) {
    int64_t nc = ncell(g);
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t f = i + g->n[0] * (j + g->n[1] * k);
                out[f] = dback(g, E, 0, i, j, k) + dback(g, E + nc, 1, i, j, k) + dback(g, E + 2 * nc, 2, i, j, k);
            }
}

void ora_div_b(const ora_grid *g, const double *B, double *out) {
    int64_t nc = ncell(g);
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t f = i + g->n[0] * (j + g->n[1] * k);
                out[f] = (fld(g, B, i + 1, j, k) - fld(g, B, i, j, k)) / g->d[0] +
                         (fld(g, B + nc, i, j + 1, k) - fld(g, B + nc, i, j, k)) / g->d[1] +
                         (fld(g, B + 2 * nc, i, j, k + 1) - fld(g, B + 2 * nc, i, j, k)) / g->d[2];
            }
}

/* ------------------------------------------------------------------ */
/* current filter                                                      */

/* One (1/4, 1/2, 1/4) pass along each axis x, y, z on each component array,
 * with the grid's boundary rule (periodic, or zero ghost beyond the x edges). */
void ora_binomial(const ora_grid *g, double *J) {
    int64_t nc = ncell(g);
    double *tmp = (double *)malloc(sizeof(double) * nc);
    for (int comp = 0; comp < 3; ++comp) {
        double *F = J + comp * nc;
        for (int ax = 0; ax < 3; ++ax) {
            for (int64_t k = 0; k < g->n[2]; ++k)
                for (int64_t j = 0; j < g->n[1]; ++j)
                    for (int64_t i = 0; i < g->n[0]; ++i) {
                        int64_t p[3] = {i, j, k}, lo[3] = {i, j, k}, hi[3] = {i, j, k};
                        lo[ax] -= 1;
                        hi[ax] += 1;
                        tmp[i + g->n[0] * (j + g->n[1] * k)] =
                            0.25 * fld(g, F, lo[0], lo[1], lo[2]) + 0.5 * fld(g, F, p[0], p[1], p[2]) +
                            0.25 * fld(g, F, hi[0], hi[1], hi[2]);
                    }
            memcpy(F, tmp, sizeof(double) * nc);
        }
    }
    free(tmp);
}

/* ------------------------------------------------------------------ */
/* coefficients of the perfect-dispersion smoothing                    */

/* Reading of Section 2: with r_y = (dx/dy)^2, r_z = (dx/dz)^2 (both <= 1 by
 * the stated constraint dx <= dy, dz):
 *   beta = (1/8, r_y/8, r_z/8); gamma_yz = r_y r_z/16, gamma_zx = r_z/16,
 *   gamma_xy = r_y/16; alpha_d = 1 - 2 beta_t1 - 2 beta_t2 - 4 gamma_{t1 t2}
 * (unit DC gain, so on-axis waves keep sigma_x = 1).  variant 1 drops the
 * corner weights (all gamma = 0), variant 2 is the identity (Yee). */
int ora_pd_coeffs(const double d[3], int variant, double alpha[3], double beta[3], double gam[3]) {
    if (d[0] <= 0 || d[1] <= 0 || d[2] <= 0) return ORA_EINVAL;
    if (variant == 2) {
        for (int a = 0; a < 3; ++a) {
            alpha[a] = 1.0;
            beta[a] = 0.0;
            gam[a] = 0.0;
        }
        return ORA_OK;
    }
    if (d[0] > d[1] || d[0] > d[2]) return ORA_EINVAL;
    double ry = (d[0] / d[1]) * (d[0] / d[1]);
    double rz = (d[0] / d[2]) * (d[0] / d[2]);
    beta[0] = 0.125;
    beta[1] = ry / 8.0;
    beta[2] = rz / 8.0;
    if (variant == 1) {
        gam[0] = gam[1] = gam[2] = 0.0;
    } else {
        gam[0] = ry * rz / 16.0;
        gam[1] = rz / 16.0;
        gam[2] = ry / 16.0;
    }
    for (int a = 0; a < 3; ++a) {
        int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
        alpha[a] = 1.0 - 2.0 * beta[t1] - 2.0 * beta[t2] - 4.0 * gam[a];
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* diagnostics                                                         */

/* out[0] = total charge q sum w dV, out[1] = field energy 1/2 sum (E^2+B^2) dV,
 * out[2] = kinetic energy m sum w (gamma - 1) dV, out[3] = max |J|. */
void ora_diag(const ora_grid *g, int64_t np, const double *u, const double *w, double q, double m,
              const double *E, const double *B, const double *J, double out[4]) {
    int64_t nc = ncell(g);
    double dv = g->d[0] * g->d[1] * g->d[2];
    double charge = 0, ef = 0, ek = 0, mj = 0;
    for (int64_t p = 0; p < np; ++p) {
        double u2 = u[p] * u[p] + u[np + p] * u[np + p] + u[2 * np + p] * u[2 * np + p];
        charge += q * w[p] * dv;
        ek += m * w[p] * (sqrt(1.0 + u2) - 1.0) * dv;
    }
    for (int64_t f = 0; f < 3 * nc; ++f) {
        ef += 0.5 * (E[f] * E[f] + B[f] * B[f]) * dv;
        if (J && fabs(J[f]) > mj) mj = fabs(J[f]);
    }
    out[0] = charge;
    out[1] = ef;
    out[2] = ek;
    out[3] = mj;
}

/* ------------------------------------------------------------------ */
/* whole step                                                          */

/* One PIC step for one species on a grid whose x boundary is periodic or
 * bounded (no window motion here).  x, u: in/out; J: out (overwritten with
 * J^{n+1/2}, after the filter when jpost == 1); E, B: in/out. x_prev (may be
 * NULL) receives x^n.  Returns ORA_ENONFINITE if a non-finite value appears. */
int ora_step(const ora_grid *g, int64_t np, double *x, double *u, const double *w, double q, double m,
             double *E, double *B, double *J, int jpost, double *x_prev) {
    int64_t nc = ncell(g);
    double *x0 = (double *)malloc(sizeof(double) * 3 * np);
    double *x1 = (double *)malloc(sizeof(double) * 3 * np);
    memcpy(x0, x, sizeof(double) * 3 * np);
    int st = ora_push(g, np, x, u, x1, q, m, E, B);
    memset(J, 0, sizeof(double) * 3 * nc);
    ora_deposit(g, np, x0, x1, w, q, J);
    if (jpost == 1) ora_binomial(g, J);
    ora_field_step(g, E, B, J);
    if (x_prev) memcpy(x_prev, x0, sizeof(double) * 3 * np);
    free(x0);
    free(x1);
    for (int64_t f = 0; f < 3 * nc && st == ORA_OK; ++f)
        if (!isfinite(E[f]) || !isfinite(B[f])) st = ORA_ENONFINITE;
    return st;
}

/* ------------------------------------------------------------------ */
/* transverse perfectly matched layer                                  */

/* Section 3.1 surrounds its Cartesian domain transversely with a 16-layer
 * perfectly matched layer.  The paper gives no formulation; this is the
 * convolutional form (stretched coordinates d/dy -> d/dy / s_y with
 * s_y = 1 + sigma_y / (i omega), kappa = 1, no frequency shift): every
 * transverse derivative term D_d F of a curl carries an auxiliary psi that
 * follows psi <- b psi + (b - 1) D_d F with b = exp(-sigma_d h) for an
 * update of time increment h, and the curl uses D_d F + psi.
 *
 * Grading: at position p (in cells, integer for nodes, half-integer for
 * face centres) along an axis of n cells with a layer of L cells,
 * depth = max((L - 1 - p) / L, (p - (n - L)) / L), clipped to [0, 1] (the
 * profile is symmetric under p -> n - 1 - p, zero on nodes L-1 .. n-L), and
 * sigma = sigma_max depth^grade.  Zero fields lie beyond the outer faces
 * (grid yzbc bits).  In normalised units (c = eps0 = 1, impedance 1)
 * sigma_max = 0.8 (grade + 1) / d is the usual choice; grade 3. */
typedef struct {
    int64_t layers;
    double sigma_max[3];   /* per axis; index 0 unused (no layer along x) */
    double grade;          /* exponent of the profile (0: constant sigma_max over the layer) */
} ora_pml;

/* sigma at position p (in cells) along axis a of n cells */
static double pml_sigma(const ora_pml *P, int a, int64_t n, double p) {
    double L = (double)P->layers;
    double lo = (L - 1.0 - p) / L, hi = (p - ((double)n - L)) / L;
    double depth = lo > hi ? lo : hi;
    if (!(depth > 0.0)) return 0.0;
    if (depth > 1.0) depth = 1.0;
    return P->sigma_max[a] * pow(depth, P->grade);
}

/* psi update and stretched derivative: returns D + psi' with psi' = b psi + (b - 1) D */
static double stretch(double *psi, double D, double sigma, double h) {
    double b = exp(-sigma * h);
    *psi = b * (*psi) + (b - 1.0) * D;
    return D + *psi;
}

/* Stretched derivative D + psi' with psi' = b psi + (b - 1) D, b = exp(-sigma dt);
 * psi' is written back when `store` is set. */
static double stretch_b(double *psi, double D, double sigma, double dt, int store) {
    double b = exp(-sigma * dt);
    double p = b * (*psi) + (b - 1.0) * D;
    if (store) *psi = p;
    return D + p;
}

/* B -= (dt/2) curl' E with the layer's stretched transverse derivatives.
 * The two half steps of B together are the leapfrog step B^{n-1/2} ->
 * B^{n+1/2} = B^{n-1/2} - dt curl' E^n, so the auxiliary arrays of B follow
 * the leapfrog recursion at the half-integer times: the first half step of a
 * step advances them with E^n (store = 1) and the second uses, without
 * storing, the value that the next step's first half step will store (the
 * same E^{n+1}).  psi[0..3]: B_x by y, B_x by z, B_y by z, B_z by y (each
 * ncell); the derivatives sit at the half-integer position of their axis. */
static void b_half_pml(const ora_grid *g, const ora_pml *P, const double *E, double *B, double *psi, int store) {
    int64_t nc = ncell(g);
    double h = 0.5 * g->dt;
    double *tmp = (double *)malloc(sizeof(double) * 3 * nc);
    const double *Ex = E, *Ey = E + nc, *Ez = E + 2 * nc;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t f = i + g->n[0] * (j + g->n[1] * k);
                double sy = pml_sigma(P, 1, g->n[1], (double)j + 0.5), sz = pml_sigma(P, 2, g->n[2], (double)k + 0.5);
                double dyEz = stretch_b(psi + f, dsmooth(g, Ez, 1, i, j, k), sy, g->dt, store);
                double dzEy = stretch_b(psi + nc + f, dsmooth(g, Ey, 2, i, j, k), sz, g->dt, store);
                double dzEx = stretch_b(psi + 2 * nc + f, dsmooth(g, Ex, 2, i, j, k), sz, g->dt, store);
                double dyEx = stretch_b(psi + 3 * nc + f, dsmooth(g, Ex, 1, i, j, k), sy, g->dt, store);
                tmp[f] = dyEz - dzEy;
                tmp[nc + f] = dzEx - dsmooth(g, Ez, 0, i, j, k);
                tmp[2 * nc + f] = dsmooth(g, Ey, 0, i, j, k) - dyEx;
            }
    for (int64_t f = 0; f < 3 * nc; ++f) B[f] -= h * tmp[f];
    free(tmp);
}

/* E += dt (curl B - J) with the layer's stretched transverse derivatives.
 * psi[0..3]: E_x by y, E_x by z, E_y by z, E_z by y; the derivatives of E's
 * update sit on the integer position of their axis. */
static void e_full_pml(const ora_grid *g, const ora_pml *P, double *E, const double *B, const double *J, double *psi) {
    int64_t nc = ncell(g);
    double *tmp = (double *)malloc(sizeof(double) * 3 * nc);
    const double *Bx = B, *By = B + nc, *Bz = B + 2 * nc;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t f = i + g->n[0] * (j + g->n[1] * k);
                double sy = pml_sigma(P, 1, g->n[1], (double)j), sz = pml_sigma(P, 2, g->n[2], (double)k);
                double dyBz = stretch(psi + f, dback(g, Bz, 1, i, j, k), sy, g->dt);
                double dzBy = stretch(psi + nc + f, dback(g, By, 2, i, j, k), sz, g->dt);
                double dzBx = stretch(psi + 2 * nc + f, dback(g, Bx, 2, i, j, k), sz, g->dt);
                double dyBx = stretch(psi + 3 * nc + f, dback(g, Bx, 1, i, j, k), sy, g->dt);
                tmp[f] = dyBz - dzBy;
                tmp[nc + f] = dzBx - dback(g, Bz, 0, i, j, k);
                tmp[2 * nc + f] = dback(g, By, 0, i, j, k) - dyBx;
            }
    for (int64_t f = 0; f < 3 * nc; ++f) E[f] += g->dt * (tmp[f] - (J ? J[f] : 0.0));
    free(tmp);
}

/* One field step with the transverse layer: psi holds 8 ncell arrays, the
 * four of the B updates then the four of the E update, carried from step
 * to step (zero at the start). */
void ora_pml_field_step(const ora_grid *g, const ora_pml *P, double *E, double *B, const double *J, double *psi) {
    int64_t nc = ncell(g);
    b_half_pml(g, P, E, B, psi, 1);
    e_full_pml(g, P, E, B, J, psi + 4 * nc);
    b_half_pml(g, P, E, B, psi, 0);
}

double ora_pml_sigma(const ora_pml *P, int a, int64_t n, double p) { return pml_sigma(P, a, n, p); }

/* ------------------------------------------------------------------ */
/* laser-wakefield boundaries: laser source, moving window, plasma     */

/* Linearly polarised (E along y) Gaussian pulse entering through the plane
 * x = src_x dx, travelling in +x.  It is built from the vector potential
 * A_y(t) = a0 env(t) cos(w0 (t - t_peak)), env = exp(-2 ln2 (t - t_peak)^2 / fwhm^2)
 * (intensity FWHM = fwhm), so E_y = -dA_y/dt has no DC part; transverse
 * profile exp(-((y-yc)^2 + (z-zc)^2) / waist^2).  The incident wave is
 * E_y(x,t) = B_z(x,t) = e(t - (x - x_src)) f(y,z). */
typedef struct {
    double a0, omega0, waist, fwhm, t_peak, t_end, yc, zc;
    int64_t src_x;
} ora_laser;

double ora_laser_e(const ora_laser *L, double t) {
    double tau = t - L->t_peak;
    double k = 2.0 * log(2.0) / (L->fwhm * L->fwhm);
    double env = exp(-k * tau * tau);
    double denv = -2.0 * k * tau * env;
    double ph = L->omega0 * tau;
    /* -d/dt [a0 env cos(ph)] */
    return -L->a0 * (denv * cos(ph) - env * L->omega0 * sin(ph));
}

double ora_laser_profile(const ora_laser *L, double y, double z) {
    double r2 = (y - L->yc) * (y - L->yc) + (z - L->zc) * (z - L->zc);
    return exp(-r2 / (L->waist * L->waist));
}

/* Total-field / scattered-field injection on the source plane: x >= x_src
 * holds the total field, x < x_src only what scatters back.  The B_z half
 * step behind the plane sees the incident E_y(x_src, t) subtracted:
 * B_z(src_x - 1/2) += h e(t) f / dx.  The E_y step on the plane sees the
 * incident B_z(x_src - dx/2, t_half) added: E_y(src_x) += dt e(t_half + dx/2) f / dx. */
void ora_laser_b_correction(const ora_grid *g, const ora_laser *L, double *B, double h, double t) {
    int64_t nc = ncell(g);
    int64_t i = L->src_x - 1;
    if (i < 0 || i >= g->n[0]) return;
    double e = ora_laser_e(L, t);
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j) {
            double f = ora_laser_profile(L, (j + 0.5) * g->d[1], k * g->d[2]);
            B[2 * nc + i + g->n[0] * (j + g->n[1] * k)] += h * e * f / g->d[0];
        }
}

void ora_laser_e_correction(const ora_grid *g, const ora_laser *L, double *E, double t_half) {
    int64_t nc = ncell(g);
    int64_t i = L->src_x;
    if (i < 0 || i >= g->n[0]) return;
    double b = ora_laser_e(L, t_half + 0.5 * g->d[0]);
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j) {
            double f = ora_laser_profile(L, (j + 0.5) * g->d[1], k * g->d[2]);
            E[nc + i + g->n[0] * (j + g->n[1] * k)] += g->dt * b * f / g->d[0];
        }
}

/* Field step of the step that starts at time t (E^n at t = n dt), with the
 * laser source applied when L is non-NULL. */
void ora_field_step_laser(const ora_grid *g, double *E, double *B, const double *J, const ora_laser *L,
                          double t) {
    b_half(g, E, B, 0.5 * g->dt);
    if (L) ora_laser_b_correction(g, L, B, 0.5 * g->dt, t);
    e_full(g, E, B, J);
    if (L) ora_laser_e_correction(g, L, E, t + 0.5 * g->dt);
    b_half(g, E, B, 0.5 * g->dt);
    if (L) ora_laser_b_correction(g, L, B, 0.5 * g->dt, t + g->dt);
}

/* The same with the transverse layer (P, psi as ora_pml_field_step). */
void ora_field_step_laser_pml(const ora_grid *g, double *E, double *B, const double *J, const ora_laser *L,
                              double t, const ora_pml *P, double *psi) {
    int64_t nc = ncell(g);
    b_half_pml(g, P, E, B, psi, 1);
    if (L) ora_laser_b_correction(g, L, B, 0.5 * g->dt, t);
    e_full_pml(g, P, E, B, J, psi + 4 * nc);
    if (L) ora_laser_e_correction(g, L, E, t + 0.5 * g->dt);
    b_half_pml(g, P, E, B, psi, 0);
    if (L) ora_laser_b_correction(g, L, B, 0.5 * g->dt, t + g->dt);
}

/* One array of ncell values moves one cell toward -x; the new leading plane is zero. */
static void shift_down_x(const ora_grid *g, double *F) {
    int64_t nx = g->n[0];
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j) {
            double *row = F + nx * (j + g->n[1] * k);
            for (int64_t i = 0; i + 1 < nx; ++i) row[i] = row[i + 1];
            row[nx - 1] = 0.0;
        }
}

/* The layer's eight auxiliary arrays move with the window like the fields. */
void ora_pml_window_shift(const ora_grid *g, double *psi) {
    int64_t nc = ncell(g);
    for (int a = 0; a < 8; ++a) shift_down_x(g, psi + a * nc);
}

/* Moving window, one cell: every field moves one cell toward -x (the plane
 * at x index 0 leaves the box) and the new leading plane is vacuum. */
void ora_window_shift(const ora_grid *g, double *E, double *B) {
    int64_t nc = ncell(g), nx = g->n[0];
    for (int comp = 0; comp < 6; ++comp) {
        double *F = comp < 3 ? E + comp * nc : B + (comp - 3) * nc;
        for (int64_t k = 0; k < g->n[2]; ++k)
            for (int64_t j = 0; j < g->n[1]; ++j) {
                double *row = F + nx * (j + g->n[1] * k);
                for (int64_t i = 0; i + 1 < nx; ++i) row[i] = row[i + 1];
                row[nx - 1] = 0.0;
            }
    }
}

/* Electron density profile along the lab-frame x (in cells): zero before
 * x_start, a linear ramp over `ramp` cells, then the plateau n_plateau. */
typedef struct {
    double x_start, ramp, n_plateau;
    int32_t ppc[3];
} ora_plasma;

double ora_density(const ora_plasma *P, double x_cells) {
    if (x_cells < P->x_start) return 0.0;
    if (P->ramp > 0.0 && x_cells < P->x_start + P->ramp) return P->n_plateau * (x_cells - P->x_start) / P->ramp;
    return P->n_plateau;
}

/* Cold plasma loading of window cells [xb, xe) when the window has moved by
 * `shift` cells: ppc[0] x ppc[1] x ppc[2] particles per cell on the sub-cell
 * lattice (k + 1/2)/ppc_d, weight n(x_lab)/ppc evaluated at each particle's
 * lab position, none where n = 0.  Tag: ((X ny + j) nz + k) ppc + s (mod 2^31),
 * X the lab cell.  Writes window positions x[3][cap], weights, tags; returns
 * the number loaded (at most cap). */
int64_t ora_inject(const ora_grid *g, const ora_plasma *P, int64_t shift, int64_t xb, int64_t xe, double *x,
                   double *w, int32_t *id, int64_t cap) {
    int64_t m = 0;
    int64_t ppc = (int64_t)P->ppc[0] * P->ppc[1] * P->ppc[2];
    for (int64_t i = xb; i < xe; ++i)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t k = 0; k < g->n[2]; ++k)
                for (int64_t s = 0; s < ppc; ++s) {
                    int64_t sx = s % P->ppc[0], sy = (s / P->ppc[0]) % P->ppc[1], sz = s / (P->ppc[0] * P->ppc[1]);
                    double ox = (sx + 0.5) / P->ppc[0], oy = (sy + 0.5) / P->ppc[1], oz = (sz + 0.5) / P->ppc[2];
                    double n = ora_density(P, (double)(shift + i) + ox);
                    if (!(n > 0.0)) continue;
                    if (m >= cap) return m;
                    x[m] = (i + ox) * g->d[0];
                    x[cap + m] = (j + oy) * g->d[1];
                    x[2 * cap + m] = (k + oz) * g->d[2];
                    w[m] = n / (double)ppc;
                    id[m] = (int32_t)((((shift + i) * g->n[1] + j) * g->n[2] + k) * ppc + s) & 0x7fffffff;
                    ++m;
                }
    return m;
}
