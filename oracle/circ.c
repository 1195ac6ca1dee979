/*
 * FP64 reference of the quasi-cylindrical particle-in-cell cycle with two
 * azimuthal modes (m = 0, 1): fields and currents decomposed into poloidal
 * modes on a (z, r) grid while the macroparticles keep their full 3D
 * Cartesian motion (Section 1; Section 3.1 uses the two lowest modes).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this code.  It shares nothing with
 * the product path; it is built into the same library as oracle.c and uses
 * its Boris rotation.
 *
 * The paper describes the method, not its discretisation.  This file takes
 * the following readings, each written from the cylindrical Maxwell
 * equations and the requirements stated beside it.
 *
 * Modes: F(r, th, z) = Re sum_m F_m(r, z) exp(-i m th), F_0 real.  The mode
 * m of a particle's charge carries exp(+i m th_p) and a factor kappa_0 = 1,
 * kappa_1 = 2 (projection (kappa_m / 2 pi) int F exp(i m th) dth).
 *
 * Grid: z nodes z_i = i dz (i < Nz), r nodes r_j = j dr (j < Nr), half nodes
 * at (i + 1/2) dz and (j + 1/2) dr.  Staggering, as (z, r):
 *   E_z (i+1/2, j), E_r (i, j+1/2), E_th (i, j)
 *   B_z (i, j+1/2), B_r (i+1/2, j), B_th (i+1/2, j+1/2); J as E; rho (i, j).
 * Arrays are [Nr][Nz], z fastest, complex.  A conducting wall at r = Nr dr
 * holds E_z = E_th = 0 there; beyond both z ends the fields are zero.
 *
 * Maxwell per mode (c = 1; d_th -> -i m):
 *   d_t B_r  =  (i m / r) E_z + d_z E_th
 *   d_t B_th = -d_z E_r + d_r E_z
 *   d_t B_z  = -(1/r) d_r (r E_th) - (i m / r) E_r
 *   d_t E_r  = -(i m / r) B_z - d_z B_th - J_r
 *   d_t E_th =  d_z B_r - d_r B_z - J_th
 *   d_t E_z  =  (1/r) d_r (r B_th) + (i m / r) B_r - J_z
 * with centred differences on the staggered grid.  On the axis (j = 0),
 * from regularity (a scalar's mode m behaves as r^m, the r and th
 * components of mode m >= 1 as r^(m-1)):
 *   m = 0: E_th = B_r = 0; E_z from the flux of B_th through the cylinder
 *          of radius dr/2: (1/r) d_r (r B_th) -> 4 B_th(dr/2) / dr;
 *   m = 1: E_z = 0; B_z is odd in r, so d_r B_z(0) = 2 B_z(dr/2) / dr;
 *          (i/r) E_z -> i d_r E_z(0) = i E_z(dr) / dr.
 * The node volumes are V_0 = pi (dr/2)^2 dz, V_j = 2 pi r_j dr dz.
 *
 * Shapes: linear in z.  In r, for the integer nodes, a particle at
 * r = (K + s) dr gives node K+1 the weight f_K(s) = s + s(1 - s)/(2(2K + 1))
 * and node K the rest: the linear weight corrected so that a uniform 3D
 * density deposits exactly n V_j on every node, the axis node included
 * (derived from that requirement; plain linear weights put 4/3 of it on the
 * axis).  Half-node components are interpolated linearly, below dr/2
 * against a ghost node at -dr/2 equal to the value at dr/2 times the mode's
 * parity (+1 for the r and th components of m = 1 and the z component of
 * m = 0, -1 otherwise).
 *
 * Gather: each mode and component at its staggered position, then
 * F = F_0 + Re(F_1 exp(-i th)) and (E_x, E_y) = (E_r cos th - E_th sin th,
 * E_r sin th + E_th cos th).  Push: relativistic Boris and a Cartesian move.
 *
 * Deposit: Esirkepov's decomposition of the change of a_i b_j c (a, b the z
 * and r shapes, c = kappa exp(i m th)) into three parts W_z, W_r, W_th
 * (symmetric weights 1, 1/2, 1/2, 1/3).  J_z and J_r are the charge fluxes
 * -(q w / dt) sum W_z (along z), -(q w / dt) sum W_r (along r) divided by
 * the node's z-face area V_j / dz and the r-face area 2 pi r_{j+1/2} dz;
 * J_th of m = 1 is -i r_j q w W_th / (V_j dt), so the discrete continuity
 * equation of each mode holds exactly at every node off the axis, and on
 * the axis for m = 0.  On the axis J_th of m = 1 is -i J_r(dr/2)
 * (regularity); J_th of m = 0, which no continuity equation fixes, is
 * deposited directly: q w v_th at the step's midpoint with the shapes there.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int64_t nz, nr;
    double dz, dr, dt;
} circ_grid;

void ora_boris(double u[3], const double Ep[3], const double Bp[3], double qm, double dt);

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- geometry */

double circ_volume(const circ_grid *g, int64_t j) {
    if (j == 0) return PI * 0.25 * g->dr * g->dr * g->dz;
    return 2.0 * PI * (double)j * g->dr * g->dr * g->dz;
}

/* ---------------------------------------------------------------- shapes */

/* Integer r nodes: base node K and weights of K, K+1 for radius r >= 0. */
void circ_shape_r(double r, double dr, int64_t *K, double w[2]) {
    double t = r / dr;
    int64_t k = (int64_t)floor(t);
    double s = t - (double)k;
    double f = s + s * (1.0 - s) / (2.0 * (2.0 * (double)k + 1.0));
    *K = k;
    w[0] = 1.0 - f;
    w[1] = f;
}

/* Linear weights for a grid with nodes at (k + sh) d: base k and two weights. */
static void lin(double x, double d, double sh, int64_t *k, double w[2]) {
    double t = x / d - sh;
    int64_t b = (int64_t)floor(t);
    double s = t - (double)b;
    *k = b;
    w[0] = 1.0 - s;
    w[1] = s;
}

/* ---------------------------------------------------------------- field access */

/* value of component array F (mode m, [nr][nz]) at (i, j); zero beyond the z ends
 * and at or beyond the wall (j >= nr) */
static cplx at(const circ_grid *g, const cplx *F, int64_t i, int64_t j) {
    if (i < 0 || i >= g->nz || j < 0 || j >= g->nr) return 0.0;
    return F[j * g->nz + i];
}

/* interpolation of an integer-r component at (z, r): z shift sz (0 or 1/2) */
static cplx interp_int(const circ_grid *g, const cplx *F, double z, double r, double sz) {
    int64_t iz, K;
    double wz[2], wr[2];
    lin(z, g->dz, sz, &iz, wz);
    circ_shape_r(r, g->dr, &K, wr);
    cplx acc = 0.0;
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) acc += wz[a] * wr[b] * at(g, F, iz + a, K + b);
    return acc;
}

/* interpolation of a half-r component at (z, r) with the mode's axis parity */
static cplx interp_half(const circ_grid *g, const cplx *F, double z, double r, double sz, double parity) {
    int64_t iz, K;
    double wz[2], wr[2];
    lin(z, g->dz, sz, &iz, wz);
    lin(r, g->dr, 0.5, &K, wr);
    cplx acc = 0.0;
    for (int b = 0; b < 2; ++b) {
        int64_t j = K + b;
        for (int a = 0; a < 2; ++a) {
            cplx v = j < 0 ? parity * at(g, F, iz + a, 0) : at(g, F, iz + a, j);
            acc += wz[a] * wr[b] * v;
        }
    }
    return acc;
}

/* ---------------------------------------------------------------- gather + push */

/* Field layout: E, B each [2 modes][3 components z, r, th][nr][nz]. */
static const cplx *comp(const circ_grid *g, const cplx *F, int m, int c) {
    return F + ((int64_t)m * 3 + c) * g->nr * g->nz;
}

/* E, B in Cartesian components at the particle position x[3] (x, y, z). */
void circ_gather(const circ_grid *g, const cplx *E, const cplx *B, const double x[3], double Ep[3], double Bp[3]) {
    double r = sqrt(x[0] * x[0] + x[1] * x[1]);
    double ct = 1.0, st = 0.0;
    if (r > 0.0) {
        ct = x[0] / r;
        st = x[1] / r;
    }
    double z = x[2];
    cplx eph = ct - I * st;   /* exp(-i th) */
    double F[2][3];          /* E, B: (z, r, th) */
    for (int f = 0; f < 2; ++f) {
        const cplx *A = f == 0 ? E : B;
        for (int c = 0; c < 3; ++c) {
            double tot = 0.0;
            for (int m = 0; m < 2; ++m) {
                const cplx *C = comp(g, A, m, c);
                cplx v;
                /* staggering: E_z (1/2, 0), E_r (0, 1/2), E_th (0, 0); B_z (0, 1/2), B_r (1/2, 0), B_th (1/2, 1/2) */
                if (f == 0) {
                    if (c == 0) v = interp_int(g, C, z, r, 0.5);
                    else if (c == 1) v = interp_half(g, C, z, r, 0.0, m == 1 ? 1.0 : -1.0);
                    else v = interp_int(g, C, z, r, 0.0);
                } else {
                    if (c == 0) v = interp_half(g, C, z, r, 0.0, m == 1 ? -1.0 : 1.0);
                    else if (c == 1) v = interp_int(g, C, z, r, 0.5);
                    else v = interp_half(g, C, z, r, 0.5, m == 1 ? 1.0 : -1.0);
                }
                tot += m == 0 ? creal(v) : creal(v * eph);
            }
            F[f][c] = tot;
        }
    }
    Ep[0] = F[0][1] * ct - F[0][2] * st;
    Ep[1] = F[0][1] * st + F[0][2] * ct;
    Ep[2] = F[0][0];
    Bp[0] = F[1][1] * ct - F[1][2] * st;
    Bp[1] = F[1][1] * st + F[1][2] * ct;
    Bp[2] = F[1][0];
}

/* Gather + Boris + Cartesian move: x[3][np] (x, y, z), u[3][np]; x_new out. */
int circ_push(const circ_grid *g, int64_t np, const double *x, double *u, double *x_new, double q, double m,
              const cplx *E, const cplx *B) {
    int bad = 0;
    for (int64_t p = 0; p < np; ++p) {
        double xp[3] = {x[p], x[np + p], x[2 * np + p]};
        double up[3] = {u[p], u[np + p], u[2 * np + p]};
        double Ep[3], Bp[3];
        circ_gather(g, E, B, xp, Ep, Bp);
        ora_boris(up, Ep, Bp, q / m, g->dt);
        double gam = sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(up[a])) bad = 1;
            u[a * np + p] = up[a];
            x_new[a * np + p] = xp[a] + g->dt * up[a] / gam;
        }
    }
    return bad ? -5 : 0;
}

/* ---------------------------------------------------------------- deposit */

/* J layout: [2 modes][3 components z, r, th][nr][nz]; J += deposit of one particle. */
static void add(const circ_grid *g, cplx *J, int m, int c, int64_t i, int64_t j, cplx v) {
    if (i < 0 || i >= g->nz || j < 0 || j >= g->nr) return;
    J[(((int64_t)m * 3 + c) * g->nr + j) * g->nz + i] += v;
}

void circ_deposit_one(const circ_grid *g, const double x0[3], const double x1[3], const double u[3], double w,
                      double q, double *Jd) {
    cplx *J = (cplx *)Jd;
    double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1]);
    double r1 = sqrt(x1[0] * x1[0] + x1[1] * x1[1]);
    /* z: linear weights of both positions on the union support of 3 integer nodes */
    int64_t i0, i1, k0, k1;
    double wa0[2], wa1[2], wb0[2], wb1[2];
    lin(x0[2], g->dz, 0.0, &i0, wa0);
    lin(x1[2], g->dz, 0.0, &i1, wa1);
    circ_shape_r(r0, g->dr, &k0, wb0);
    circ_shape_r(r1, g->dr, &k1, wb1);
    int64_t bz = i0 < i1 ? i0 : i1, br = k0 < k1 ? k0 : k1;
    double a0[3] = {0, 0, 0}, a1[3] = {0, 0, 0}, b0[3] = {0, 0, 0}, b1[3] = {0, 0, 0};
    for (int t = 0; t < 2; ++t) {
        a0[i0 - bz + t] += wa0[t];
        a1[i1 - bz + t] += wa1[t];
        b0[k0 - br + t] += wb0[t];
        b1[k1 - br + t] += wb1[t];
    }
    double da[3], db[3];
    for (int t = 0; t < 3; ++t) {
        da[t] = a1[t] - a0[t];
        db[t] = b1[t] - b0[t];
    }
    double th0c = 1.0, th0s = 0.0, th1c = 1.0, th1s = 0.0;
    if (r0 > 0.0) {
        th0c = x0[0] / r0;
        th0s = x0[1] / r0;
    }
    if (r1 > 0.0) {
        th1c = x1[0] / r1;
        th1s = x1[1] / r1;
    }
    for (int m = 0; m < 2; ++m) {
        double kap = m == 0 ? 1.0 : 2.0;
        cplx c0 = m == 0 ? 1.0 : kap * (th0c + I * th0s);   /* kappa exp(i m th) */
        cplx c1 = m == 0 ? 1.0 : kap * (th1c + I * th1s);
        cplx dc = c1 - c0;
        for (int jj = 0; jj < 3; ++jj) {
            int64_t j = br + jj;
            /* J_z: flux along z, running sum over the z support */
            cplx run = 0.0;
            for (int ii = 0; ii < 3; ++ii) {
                cplx wz = da[ii] * (b0[jj] * c0 + 0.5 * db[jj] * c0 + 0.5 * b0[jj] * dc + db[jj] * dc / 3.0);
                run += wz;
                double area = circ_volume(g, j) / g->dz;
                add(g, J, m, 0, bz + ii, j, -q * w * run / (g->dt * area));
            }
        }
        for (int ii = 0; ii < 3; ++ii) {
            int64_t i = bz + ii;
            cplx run = 0.0;
            for (int jj = 0; jj < 3; ++jj) {
                int64_t j = br + jj;
                cplx wr = db[jj] * (a0[ii] * c0 + 0.5 * da[ii] * c0 + 0.5 * a0[ii] * dc + da[ii] * dc / 3.0);
                run += wr;
                double area = 2.0 * PI * ((double)j + 0.5) * g->dr * g->dz;
                add(g, J, m, 1, i, j, -q * w * run / (g->dt * area));
            }
        }
        if (m == 1) {
            for (int jj = 0; jj < 3; ++jj) {
                int64_t j = br + jj;
                if (j == 0) continue;
                for (int ii = 0; ii < 3; ++ii) {
                    cplx wt = dc * (a0[ii] * b0[jj] + 0.5 * da[ii] * b0[jj] + 0.5 * a0[ii] * db[jj] +
                                    da[ii] * db[jj] / 3.0);
                    double rj = (double)j * g->dr;
                    add(g, J, 1, 2, bz + ii, j, -I * rj * q * w * wt / (circ_volume(g, j) * g->dt));
                }
            }
        }
    }
    /* m = 0 azimuthal current at the midpoint */
    double xm[3] = {0.5 * (x0[0] + x1[0]), 0.5 * (x0[1] + x1[1]), 0.5 * (x0[2] + x1[2])};
    double rm = sqrt(xm[0] * xm[0] + xm[1] * xm[1]);
    if (rm > 0.0) {
        double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double vth = (-xm[1] * u[0] + xm[0] * u[1]) / (rm * gam);
        int64_t iz, K;
        double wz[2], wr[2];
        lin(xm[2], g->dz, 0.0, &iz, wz);
        circ_shape_r(rm, g->dr, &K, wr);
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                add(g, J, 0, 2, iz + a, K + b, q * w * vth * wz[a] * wr[b] / circ_volume(g, K + b));
    }
}

/* J += deposit of all particles (x0 -> x1 with momentum u^{n+1/2}); then the axis rule of m = 1 J_th. */
void circ_deposit(const circ_grid *g, int64_t np, const double *x0, const double *x1, const double *u,
                  const double *w, double q, double *Jd) {
    cplx *J = (cplx *)Jd;
    for (int64_t p = 0; p < np; ++p) {
        double a[3] = {x0[p], x0[np + p], x0[2 * np + p]};
        double b[3] = {x1[p], x1[np + p], x1[2 * np + p]};
        double up[3] = {u[p], u[np + p], u[2 * np + p]};
        circ_deposit_one(g, a, b, up, w[p], q, Jd);
    }
    int64_t nz = g->nz, nr = g->nr;
    cplx *Jt1 = J + (1 * 3 + 2) * nr * nz;
    const cplx *Jr1 = J + (1 * 3 + 1) * nr * nz;
    for (int64_t i = 0; i < nz; ++i) Jt1[i] = -I * Jr1[i];
}

/* Mode charge densities rho_m = sum q w kappa a_i b_j exp(i m th) / V_j, [2][nr][nz]. */
void circ_rho(const circ_grid *g, int64_t np, const double *x, const double *w, double q, double *rhod) {
    cplx *rho = (cplx *)rhod;
    for (int64_t p = 0; p < np; ++p) {
        double xx = x[p], yy = x[np + p], zz = x[2 * np + p];
        double r = sqrt(xx * xx + yy * yy);
        double ct = 1.0, st = 0.0;
        if (r > 0.0) {
            ct = xx / r;
            st = yy / r;
        }
        int64_t iz, K;
        double wz[2], wr[2];
        lin(zz, g->dz, 0.0, &iz, wz);
        circ_shape_r(r, g->dr, &K, wr);
        for (int m = 0; m < 2; ++m) {
            cplx c = m == 0 ? 1.0 : 2.0 * (ct + I * st);
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    int64_t i = iz + a, j = K + b;
                    if (i < 0 || i >= g->nz || j < 0 || j >= g->nr) continue;
                    rho[((int64_t)m * g->nr + j) * g->nz + i] += q * w[p] * wz[a] * wr[b] * c / circ_volume(g, j);
                }
        }
    }
}

/* Discrete divergence of a vector field (E or J layout) per mode on the
 * integer nodes (i, j): out [2][nr][nz]. */
void circ_div(const circ_grid *g, const double *Fd, double *outd) {
    const cplx *F = (const cplx *)Fd;
    cplx *out = (cplx *)outd;
    for (int m = 0; m < 2; ++m) {
        const cplx *Fz = comp(g, F, m, 0), *Fr = comp(g, F, m, 1), *Ft = comp(g, F, m, 2);
        for (int64_t j = 0; j < g->nr; ++j)
            for (int64_t i = 0; i < g->nz; ++i) {
                double V = circ_volume(g, j);
                cplx s = (V / g->dz) * (at(g, Fz, i, j) - at(g, Fz, i - 1, j));
                double ap = 2.0 * PI * ((double)j + 0.5) * g->dr * g->dz;
                double am = 2.0 * PI * ((double)j - 0.5) * g->dr * g->dz;
                s += ap * at(g, Fr, i, j);
                if (j > 0) s -= am * at(g, Fr, i, j - 1);
                s /= V;
                if (j > 0) s -= I * (double)m / ((double)j * g->dr) * at(g, Ft, i, j);
                out[((int64_t)m * g->nr + j) * g->nz + i] = s;
            }
    }
}

/* ---------------------------------------------------------------- field update */

/* B -= h curl E, per mode, on the staggered grid with the axis rules. */
static void b_half(const circ_grid *g, const cplx *E, cplx *B, double h) {
    int64_t nz = g->nz, nr = g->nr, N = nz * nr;
    cplx *tmp = (cplx *)calloc((size_t)(6 * N), sizeof(cplx));
    for (int m = 0; m < 2; ++m) {
        const cplx *Ez = comp(g, E, m, 0), *Er = comp(g, E, m, 1), *Et = comp(g, E, m, 2);
        cplx *tz = tmp + (m * 3 + 0) * N, *tr = tmp + (m * 3 + 1) * N, *tt = tmp + (m * 3 + 2) * N;
        for (int64_t j = 0; j < nr; ++j)
            for (int64_t i = 0; i < nz; ++i) {
                int64_t f = j * nz + i;
                double rh = ((double)j + 0.5) * g->dr;
                /* (curl E)_z at (i, j+1/2) = (1/r) d_r (r E_th) + (i m / r) E_r */
                tz[f] = (((double)(j + 1) * g->dr) * at(g, Et, i, j + 1) - ((double)j * g->dr) * at(g, Et, i, j)) /
                            (rh * g->dr) +
                        I * (double)m / rh * at(g, Er, i, j);
                /* (curl E)_r at (i+1/2, j) = -(i m / r) E_z - d_z E_th */
                if (j == 0) {
                    tr[f] = m == 0 ? 0.0
                                   : -I * at(g, Ez, i, 1) / g->dr - (at(g, Et, i + 1, 0) - at(g, Et, i, 0)) / g->dz;
                } else {
                    tr[f] = -I * (double)m / ((double)j * g->dr) * at(g, Ez, i, j) -
                            (at(g, Et, i + 1, j) - at(g, Et, i, j)) / g->dz;
                }
                /* (curl E)_th at (i+1/2, j+1/2) = d_z E_r - d_r E_z */
                tt[f] = (at(g, Er, i + 1, j) - at(g, Er, i, j)) / g->dz - (at(g, Ez, i, j + 1) - at(g, Ez, i, j)) / g->dr;
            }
    }
    for (int m = 0; m < 2; ++m)
        for (int c = 0; c < 3; ++c) {
            cplx *Bc = B + (m * 3 + c) * N;
            const cplx *t = tmp + (m * 3 + c) * N;
            for (int64_t f = 0; f < N; ++f) Bc[f] -= h * t[f];
        }
    /* m = 0: B_r on the axis stays zero */
    for (int64_t i = 0; i < nz; ++i) B[(0 * 3 + 1) * N + i] = 0.0;
    free(tmp);
}

/* E += dt (curl B - J), per mode, with the axis rules. */
static void e_full(const circ_grid *g, cplx *E, const cplx *B, const cplx *J) {
    int64_t nz = g->nz, nr = g->nr, N = nz * nr;
    cplx *tmp = (cplx *)calloc((size_t)(6 * N), sizeof(cplx));
    for (int m = 0; m < 2; ++m) {
        const cplx *Bz = comp(g, B, m, 0), *Br = comp(g, B, m, 1), *Bt = comp(g, B, m, 2);
        cplx *tz = tmp + (m * 3 + 0) * N, *tr = tmp + (m * 3 + 1) * N, *tt = tmp + (m * 3 + 2) * N;
        for (int64_t j = 0; j < nr; ++j)
            for (int64_t i = 0; i < nz; ++i) {
                int64_t f = j * nz + i;
                double rh = ((double)j + 0.5) * g->dr;
                /* (curl B)_z at (i+1/2, j) = (1/r) d_r (r B_th) + (i m / r) B_r */
                if (j == 0) {
                    tz[f] = m == 0 ? 4.0 * at(g, Bt, i, 0) / g->dr : 0.0;
                } else {
                    double rj = (double)j * g->dr;
                    tz[f] = (rh * at(g, Bt, i, j) - (rh - g->dr) * at(g, Bt, i, j - 1)) / (rj * g->dr) +
                            I * (double)m / rj * at(g, Br, i, j);
                }
                /* (curl B)_r at (i, j+1/2) = -(i m / r) B_z - d_z B_th */
                tr[f] = -I * (double)m / rh * at(g, Bz, i, j) - (at(g, Bt, i, j) - at(g, Bt, i - 1, j)) / g->dz;
                /* (curl B)_th at (i, j) = d_z B_r - d_r B_z */
                if (j == 0) {
                    tt[f] = m == 0 ? 0.0 : (at(g, Br, i, 0) - at(g, Br, i - 1, 0)) / g->dz - 2.0 * at(g, Bz, i, 0) / g->dr;
                } else {
                    tt[f] = (at(g, Br, i, j) - at(g, Br, i - 1, j)) / g->dz - (at(g, Bz, i, j) - at(g, Bz, i, j - 1)) / g->dr;
                }
            }
    }
    for (int m = 0; m < 2; ++m)
        for (int c = 0; c < 3; ++c) {
            cplx *Ec = E + (m * 3 + c) * N;
            const cplx *t = tmp + (m * 3 + c) * N;
            const cplx *Jc = J ? J + (m * 3 + c) * N : NULL;
            for (int64_t f = 0; f < N; ++f) Ec[f] += g->dt * (t[f] - (Jc ? Jc[f] : 0.0));
        }
    /* axis: E_th, E_z of the mode that cannot carry them stay zero */
    for (int64_t i = 0; i < nz; ++i) {
        E[(0 * 3 + 2) * N + i] = 0.0;   /* m = 0 E_th */
        E[(1 * 3 + 0) * N + i] = 0.0;   /* m = 1 E_z */
    }
    free(tmp);
}

/* ---------------------------------------------------------------- laser on mode 1 */

typedef struct {
    double a0, omega0, waist, fwhm, t_peak, t_end;
    int64_t src;
} circ_laser;

static double laser_e(const circ_laser *L, double t) {
    double tau = t - L->t_peak;
    double k = 2.0 * log(2.0) / (L->fwhm * L->fwhm);
    double env = exp(-k * tau * tau);
    double denv = -2.0 * k * tau * env;
    double ph = L->omega0 * tau;
    return -L->a0 * (denv * cos(ph) - env * L->omega0 * sin(ph));
}

/* A pulse linearly polarised along x, E_x = B_y = e(t - (z - z_src)) exp(-r^2/w^2):
 * mode 1 with E_r = e f, E_th = -i e f, B_r = i e f, B_th = e f.  Total-field /
 * scattered-field corrections on the B planes behind the source (src - 1/2)
 * and on the E planes on it (src). */
static void laser_b(const circ_grid *g, const circ_laser *L, cplx *B, double h, double t) {
    int64_t i = L->src - 1, N = g->nz * g->nr;
    if (i < 0 || i >= g->nz) return;
    double e = laser_e(L, t);
    for (int64_t j = 0; j < g->nr; ++j) {
        double rj = (double)j * g->dr, rh = ((double)j + 0.5) * g->dr;
        double fj = exp(-rj * rj / (L->waist * L->waist)), fh = exp(-rh * rh / (L->waist * L->waist));
        B[(1 * 3 + 2) * N + j * g->nz + i] += h * e * fh / g->dz;
        B[(1 * 3 + 1) * N + j * g->nz + i] += I * h * e * fj / g->dz;
    }
}

static void laser_e_plane(const circ_grid *g, const circ_laser *L, cplx *E, double t_half) {
    int64_t i = L->src, N = g->nz * g->nr;
    if (i < 0 || i >= g->nz) return;
    double b = laser_e(L, t_half + 0.5 * g->dz);
    for (int64_t j = 0; j < g->nr; ++j) {
        double rj = (double)j * g->dr, rh = ((double)j + 0.5) * g->dr;
        double fj = exp(-rj * rj / (L->waist * L->waist)), fh = exp(-rh * rh / (L->waist * L->waist));
        E[(1 * 3 + 1) * N + j * g->nz + i] += g->dt * b * fh / g->dz;
        E[(1 * 3 + 2) * N + j * g->nz + i] += -I * g->dt * b * fj / g->dz;
    }
}

/* One field step from time t: B half step, E step, B half step (laser if L). */
void circ_field_step(const circ_grid *g, double *Ed, double *Bd, const double *Jd, const circ_laser *L, double t) {
    cplx *E = (cplx *)Ed, *B = (cplx *)Bd;
    const cplx *J = (const cplx *)Jd;
    b_half(g, E, B, 0.5 * g->dt);
    if (L) laser_b(g, L, B, 0.5 * g->dt, t);
    e_full(g, E, B, J);
    if (L) laser_e_plane(g, L, E, t + 0.5 * g->dt);
    b_half(g, E, B, 0.5 * g->dt);
    if (L) laser_b(g, L, B, 0.5 * g->dt, t + g->dt);
}

/* Moving window: every field moves one z cell toward -z; the new front plane is zero. */
void circ_window_shift(const circ_grid *g, double *Ed, double *Bd) {
    for (int f = 0; f < 2; ++f) {
        cplx *F = (cplx *)(f == 0 ? Ed : Bd);
        for (int64_t row = 0; row < 6 * g->nr; ++row) {
            cplx *R = F + row * g->nz;
            for (int64_t i = 0; i + 1 < g->nz; ++i) R[i] = R[i + 1];
            R[g->nz - 1] = 0.0;
        }
    }
}

/* Field energy: sum over nodes of V (|F_0|^2 + |F_1|^2 / 2) / 2 per component,
 * each at its own staggered radius (half-node volumes 2 pi r_{j+1/2} dr dz). */
double circ_field_energy(const circ_grid *g, const double *Ed, const double *Bd) {
    int64_t N = g->nz * g->nr;
    double e = 0.0;
    /* integer-r components: E_z, E_th, B_r; half-r: E_r, B_z, B_th */
    const int half_e[3] = {0, 1, 0}, half_b[3] = {1, 0, 1};
    for (int f = 0; f < 2; ++f) {
        const cplx *F = (const cplx *)(f == 0 ? Ed : Bd);
        for (int m = 0; m < 2; ++m)
            for (int c = 0; c < 3; ++c) {
                int half = f == 0 ? half_e[c] : half_b[c];
                const cplx *C = F + (m * 3 + c) * N;
                for (int64_t j = 0; j < g->nr; ++j) {
                    double V = half ? 2.0 * PI * ((double)j + 0.5) * g->dr * g->dr * g->dz : circ_volume(g, j);
                    for (int64_t i = 0; i < g->nz; ++i) {
                        double a = cabs(C[j * g->nz + i]);
                        e += 0.5 * V * a * a * (m == 0 ? 1.0 : 0.5);
                    }
                }
            }
    }
    return e;
}
