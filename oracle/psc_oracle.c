/*
 * psc_oracle.c -- plain double-precision reference of the explicit
 * electromagnetic particle-in-cell timestep of Germaschewski et al.,
 * "The Plasma Simulation Code" (J. Comput. Phys., arXiv 1310.7866).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code,
 * header, table or helper with the HIP library; it is written to be read
 * against the paper, not to be fast.
 *
 * What it computes (every routine cites the passage it follows):
 *   - Yee staggered grid and the discrete curls/divergences (sec. "FDTD
 *     method for solving Maxwell's equations", eqs. for nabla^+ x E,
 *     nabla^- x B, nabla^+ . B, nabla^- . E);
 *   - the leap-frog field update split as in the optimized time step
 *     (fig. psc_new): B half step, particle loop, B half step, E full step;
 *   - B-spline shape functions b1, b2 (sec. "Time integration of the
 *     quasi-particle equations of motion", B-spline definitions), used as
 *     interpolation weights one order above the particle shape (eq.
 *     E_interp and the remark that follows the b1/b2 definitions);
 *   - the relativistic Boris push (same section, Boris' splitting);
 *   - Esirkepov's charge-conserving current deposit (sec. "Time
 *     integration", charge continuity), written from the discrete
 *     continuity equation rho^{n+1/2} - rho^{n-1/2} + dt div^- j = 0;
 *   - the Villasenor-Buneman deposit the paper uses for 1st-order
 *     particles (same section), by cutting the path at cell faces;
 *   - Marder's divergence cleaning step (same section);
 *   - a stable sort of particles by a patch-major cell key (sec. "Sorting
 *     and Communication").
 *
 * Conventions (readings where the paper fixes no units): c = eps0 = 1;
 * dE/dt = curl B - J; dB/dt = -curl E; du/dt = (q/m)(E + u x B / gamma);
 * positions are absolute, in cell units (xi = x / dx); a 2-d grid is the
 * (y, z) plane with n[0] == 1 and no x derivatives.  Field arrays are component-major, index i + n0*(j + n1*k).
 *
 * Parity status: every routine is pinned by a closed form, an identity or
 * brute force in the CPU tests, except the out-of-plane current J_x of the
 * 2-d deposit for cell-crossing moves (pinned only for moves inside one
 * cell, where it equals the exact time average of the shape).  The energy
 * diagnostics are pinned by closed forms (rational gamma, uniform fields)
 * and by the energy balance of the cold plasma oscillation; the energy of
 * a general run has no exact value (the scheme does not conserve it).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Built with OpenMP (only for timing the oracle on all host cores), the
 * particle loop and the field updates run in parallel threads; each thread
 * deposits into its own copy of J, and the copies are added in thread
 * order.  The default build (the tests' reference) has no threads. */
/* Threads of the parallel loops (1 without OpenMP); returns the count. */
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

typedef struct {
    int dim;        /* 2: (y,z) plane, x invariant; 3: (x,y,z)          */
    int n[3];       /* cells along x, y, z                              */
    double d[3];    /* cell sizes                                       */
    double dt;      /* time step                                        */
    int order;      /* 1: b1 weights, 2: b2 weights                     */
    int vb;         /* 1st order: Villasenor-Buneman deposit instead of Esirkepov */
} orc_grid;

/* ----------------------------------------------------------------------- */
/* grid helpers                                                            */
/* ----------------------------------------------------------------------- */

static int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

static long idx3(const orc_grid *g, int i, int j, int k) {
    return (long)wrapi(i, g->n[0]) + (long)g->n[0] * ((long)wrapi(j, g->n[1]) + (long)g->n[1] * wrapi(k, g->n[2]));
}

static long ncell(const orc_grid *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static int active(const orc_grid *g, int d) { return g->dim == 3 || d > 0; }

/* Staggering (in cells) of each component on the Yee cell (fig. grid and the
 * component lists E_ijk, B_ijk): E on edges, B on faces. */
static const double STAG_E[3][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
static const double STAG_B[3][3] = {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

/* ----------------------------------------------------------------------- */
/* B-splines                                                               */
/* ----------------------------------------------------------------------- */

/* b1 and b2 exactly as printed after the recursive definition b_{n+1} = b0 (*) b_n. */
double orc_bspline(int order, double s) {
    double a = fabs(s);
    if (order == 0) return a < 0.5 ? 1.0 : 0.0;
    if (order == 1) return a <= 1.0 ? 1.0 - a : 0.0;
    if (a <= 0.5) return 0.75 - a * a;
    if (a <= 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

/* ----------------------------------------------------------------------- */
/* Interpolation (eq. E_interp): F_p = sum_nodes b(xi - node) F(node)        */
/* ----------------------------------------------------------------------- */

double orc_interp(const orc_grid *g, const double *F, const double xi[3], const double stag[3]) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        if (!active(g, d)) continue;
        lo[d] = (int)floor(xi[d] - stag[d]) - 2;   /* window wider than any support */
        hi[d] = lo[d] + 5;
    }
    double sum = 0.0;
    for (int k = lo[2]; k <= hi[2]; ++k) {
        double wz = active(g, 2) ? orc_bspline(g->order, xi[2] - stag[2] - k) : 1.0;
        if (wz == 0.0) continue;
        for (int j = lo[1]; j <= hi[1]; ++j) {
            double wy = active(g, 1) ? orc_bspline(g->order, xi[1] - stag[1] - j) : 1.0;
            if (wy == 0.0) continue;
            for (int i = lo[0]; i <= hi[0]; ++i) {
                double wx = active(g, 0) ? orc_bspline(g->order, xi[0] - stag[0] - i) : 1.0;
                if (wx == 0.0) continue;
                sum += wx * wy * wz * F[idx3(g, i, j, k)];
            }
        }
    }
    return sum;
}

/* ----------------------------------------------------------------------- */
/* Boris push (Boris' split: half E kick, rotation by B, half E kick)       */
/* ----------------------------------------------------------------------- */

void orc_boris(double u[3], const double E[3], const double B[3], double qdt_2m) {
    double um[3], t[3], s[3], up[3], uq[3];
    for (int c = 0; c < 3; ++c) um[c] = u[c] + qdt_2m * E[c];
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int c = 0; c < 3; ++c) t[c] = qdt_2m * B[c] / gm;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int c = 0; c < 3; ++c) s[c] = 2.0 * t[c] / (1.0 + t2);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    uq[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
    uq[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
    uq[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
    for (int c = 0; c < 3; ++c) u[c] = uq[c] + qdt_2m * E[c];
}

/* ----------------------------------------------------------------------- */
/* Esirkepov deposit: current of one particle moving xi0 -> xi1 (unwrapped) */
/* ----------------------------------------------------------------------- */

#define ESK 6   /* stencil nodes per dimension: covers both supports at order <= 2 */

/* Adds the particle's current density to J (3 component arrays).  qw is the
 * charge times density weight, vx the out-of-plane velocity used in 2-d. */
void orc_deposit(const orc_grid *g, double *J, const double xi0[3], const double xi1[3],
                 double qw, double vx) {
    double S0[3][ESK], DS[3][ESK];
    int base[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        for (int l = 0; l < ESK; ++l) { S0[d][l] = 0.0; DS[d][l] = 0.0; }
        if (!active(g, d)) { S0[d][0] = 1.0; continue; }
        base[d] = (int)floor(xi0[d]) - 2;
        for (int l = 0; l < ESK; ++l) {
            double node = base[d] + l;
            S0[d][l] = orc_bspline(g->order, xi0[d] - node);
            DS[d][l] = orc_bspline(g->order, xi1[d] - node) - S0[d][l];
        }
    }
    long nc = ncell(g);
    double *Jx = J, *Jy = J + nc, *Jz = J + 2 * nc;
    const double third = 1.0 / 3.0;
    if (g->dim == 3) {
        double fx = -qw * g->d[0] / g->dt, fy = -qw * g->d[1] / g->dt, fz = -qw * g->d[2] / g->dt;
        for (int n = 0; n < ESK; ++n)
            for (int m = 0; m < ESK; ++m) {
                double acc = 0.0;   /* running sum along x */
                for (int l = 0; l < ESK; ++l) {
                    double W = DS[0][l] * (S0[1][m] * S0[2][n] + 0.5 * DS[1][m] * S0[2][n] +
                                           0.5 * S0[1][m] * DS[2][n] + third * DS[1][m] * DS[2][n]);
                    acc += W;
                    Jx[idx3(g, base[0] + l, base[1] + m, base[2] + n)] += fx * acc;
                }
            }
        for (int n = 0; n < ESK; ++n)
            for (int l = 0; l < ESK; ++l) {
                double acc = 0.0;
                for (int m = 0; m < ESK; ++m) {
                    double W = DS[1][m] * (S0[0][l] * S0[2][n] + 0.5 * DS[0][l] * S0[2][n] +
                                           0.5 * S0[0][l] * DS[2][n] + third * DS[0][l] * DS[2][n]);
                    acc += W;
                    Jy[idx3(g, base[0] + l, base[1] + m, base[2] + n)] += fy * acc;
                }
            }
        for (int m = 0; m < ESK; ++m)
            for (int l = 0; l < ESK; ++l) {
                double acc = 0.0;
                for (int n = 0; n < ESK; ++n) {
                    double W = DS[2][n] * (S0[0][l] * S0[1][m] + 0.5 * DS[0][l] * S0[1][m] +
                                           0.5 * S0[0][l] * DS[1][m] + third * DS[0][l] * DS[1][m]);
                    acc += W;
                    Jz[idx3(g, base[0] + l, base[1] + m, base[2] + n)] += fz * acc;
                }
            }
    } else {
        double fy = -qw * g->d[1] / g->dt, fz = -qw * g->d[2] / g->dt;
        for (int n = 0; n < ESK; ++n) {
            double acc = 0.0;
            for (int m = 0; m < ESK; ++m) {
                acc += DS[1][m] * (S0[2][n] + 0.5 * DS[2][n]);
                Jy[idx3(g, 0, base[1] + m, base[2] + n)] += fy * acc;
            }
        }
        for (int m = 0; m < ESK; ++m) {
            double acc = 0.0;
            for (int n = 0; n < ESK; ++n) {
                acc += DS[2][n] * (S0[1][m] + 0.5 * DS[1][m]);
                Jz[idx3(g, 0, base[1] + m, base[2] + n)] += fz * acc;
            }
        }
        for (int n = 0; n < ESK; ++n)
            for (int m = 0; m < ESK; ++m) {
                double sh = S0[1][m] * S0[2][n] + 0.5 * DS[1][m] * S0[2][n] +
                            0.5 * S0[1][m] * DS[2][n] + third * DS[1][m] * DS[2][n];
                Jx[idx3(g, 0, base[1] + m, base[2] + n)] += qw * vx * sh;
            }
    }
}

/* ----------------------------------------------------------------------- */
/* Villasenor-Buneman deposit (1st order; the paper's charge-conserving     */
/* scheme for 1st-order particles, sec. "Time integration")                 */
/* ----------------------------------------------------------------------- */

/* The straight path xi0 -> xi1 is cut at the cell faces it crosses.  A piece
 * inside one cell moves a linear (area in 2-d, volume in 3-d) charge cloud;
 * the current through each edge of that cell is the cloud's flux: along x,
 * q w dx/dt times the time average over the piece of the product of the
 * linear weights in the other directions, which for straight motion is the
 * product at the piece's midpoint plus (+/-) the product of the other two
 * displacements over 12 (3-d).  In 2-d the out-of-plane current is
 * q w v_x times the piece's share of the step times the linear weights at
 * its midpoint. */
void orc_deposit_vb(const orc_grid *g, double *J, const double xi0[3], const double xi1[3],
                    double qw, double vx) {
    double t[5];
    int nt = 0;
    t[nt++] = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (!active(g, d)) continue;
        double a = xi0[d], b = xi1[d];
        double fa = floor(a), fb = floor(b);
        if (fa != fb) {                          /* one face between them (|b - a| < 1) */
            double face = fb > fa ? fb : fa;
            t[nt++] = (face - a) / (b - a);
        }
    }
    t[nt++] = 1.0;
    for (int i = 1; i < nt; ++i)                 /* sort the cut parameters */
        for (int k = i; k > 0 && t[k] < t[k - 1]; --k) {
            double x = t[k]; t[k] = t[k - 1]; t[k - 1] = x;
        }
    long nc = ncell(g);
    double *Jx = J, *Jy = J + nc, *Jz = J + 2 * nc;
    for (int p = 0; p + 1 < nt; ++p) {
        double ta = t[p], tb = t[p + 1];
        if (!(tb > ta)) continue;
        int c[3] = {0, 0, 0};
        double m[3] = {0, 0, 0}, dd[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            if (!active(g, d)) continue;
            double pa = xi0[d] + ta * (xi1[d] - xi0[d]), pb = xi0[d] + tb * (xi1[d] - xi0[d]);
            double mid = 0.5 * (pa + pb);
            c[d] = (int)floor(mid);
            m[d] = mid - c[d];
            dd[d] = pb - pa;
        }
        /* linear weights of the midpoint at the cell's lower (0) and upper (1) node */
        double w[3][2];
        for (int d = 0; d < 3; ++d) { w[d][0] = 1.0 - m[d]; w[d][1] = m[d]; }
        if (g->dim == 3) {
            double fx = qw * g->d[0] / g->dt, fy = qw * g->d[1] / g->dt, fz = qw * g->d[2] / g->dt;
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e) {
                    double sg = (b == e) ? 1.0 : -1.0;
                    Jx[idx3(g, c[0], c[1] + b, c[2] + e)] += fx * dd[0] * (w[1][b] * w[2][e] + sg * dd[1] * dd[2] / 12.0);
                    Jy[idx3(g, c[0] + b, c[1], c[2] + e)] += fy * dd[1] * (w[0][b] * w[2][e] + sg * dd[0] * dd[2] / 12.0);
                    Jz[idx3(g, c[0] + b, c[1] + e, c[2])] += fz * dd[2] * (w[0][b] * w[1][e] + sg * dd[0] * dd[1] / 12.0);
                }
        } else {
            double fy = qw * g->d[1] / g->dt, fz = qw * g->d[2] / g->dt;
            for (int e = 0; e < 2; ++e) {
                Jy[idx3(g, 0, c[1], c[2] + e)] += fy * dd[1] * w[2][e];
                Jz[idx3(g, 0, c[1] + e, c[2])] += fz * dd[2] * w[1][e];
            }
            for (int e = 0; e < 2; ++e)
                for (int b = 0; b < 2; ++b)
                    Jx[idx3(g, 0, c[1] + b, c[2] + e)] += qw * vx * (tb - ta) * w[1][b] * w[2][e];
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Particle loop (fig. psc_new: push_particle_p, push_particle_x, deposit_j) */
/* ----------------------------------------------------------------------- */

/* One particle p of the loop below: gather E and B at its position, Boris
 * push, move, deposit its current into J. */
static void push_particle(const orc_grid *g, long np, long p, double *xi, double *u, const double *E,
                          const double *B, double *J, double q, double m, double w) {
    long nc = ncell(g);
    double qdt_2m = q * g->dt / (2.0 * m);
    double x0[3], x1[3], uu[3], Ep[3], Bp[3];
    for (int d = 0; d < 3; ++d) { x0[d] = xi[d * np + p]; uu[d] = u[d * np + p]; }
    for (int c = 0; c < 3; ++c) {
        Ep[c] = orc_interp(g, E + c * nc, x0, STAG_E[c]);
        Bp[c] = orc_interp(g, B + c * nc, x0, STAG_B[c]);
    }
    orc_boris(uu, Ep, Bp, qdt_2m);
    double gam = sqrt(1.0 + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
    for (int d = 0; d < 3; ++d)
        x1[d] = active(g, d) ? x0[d] + g->dt * uu[d] / (gam * g->d[d]) : x0[d];
    if (g->vb) orc_deposit_vb(g, J, x0, x1, q * w, uu[0] / gam);
    else orc_deposit(g, J, x0, x1, q * w, uu[0] / gam);
    for (int d = 0; d < 3; ++d) {
        double x = x1[d];
        if (active(g, d)) {
            if (x < 0.0) x += g->n[d];
            if (x >= g->n[d]) x -= g->n[d];
            if (x >= g->n[d]) x -= g->n[d];   /* -tiny + n rounded to n */
        }
        xi[d * np + p] = x;
        u[d * np + p] = uu[d];
    }
}

/* xi: (3, n) absolute positions in cells at t^{n+1/2}; u: (3, n) at t^n.
 * E at t^{n+1/2}, B at t^{n+1/2}; J accumulates (not cleared here).
 * On return xi holds t^{n+3/2} (wrapped into [0, n_d)) and u holds t^{n+1}. */
void orc_push_particles(const orc_grid *g, long np, double *xi, double *u,
                        const double *E, const double *B, double *J,
                        double q, double m, double w) {
#ifdef _OPENMP
    int nt = omp_get_max_threads();
    size_t len = 3 * (size_t)ncell(g);
    double *Jt = nt > 1 ? (double *)malloc((size_t)nt * len * sizeof(double)) : NULL;
    if (Jt) {
        int team = 1;
#pragma omp parallel num_threads(nt)
        {
            double *Jp = Jt + (size_t)omp_get_thread_num() * len;
            memset(Jp, 0, len * sizeof(double));
#pragma omp single
            team = omp_get_num_threads();   /* copies in use (the barrier follows) */
#pragma omp for schedule(static)
            for (long p = 0; p < np; ++p) push_particle(g, np, p, xi, u, E, B, Jp, q, m, w);
#pragma omp for schedule(static)
            for (long i = 0; i < (long)len; ++i) {
                double a = 0.0;
                for (int t = 0; t < team; ++t) a += Jt[(size_t)t * len + i];
                J[i] += a;
            }
        }
        free(Jt);
        return;
    }
#endif
    for (long p = 0; p < np; ++p) push_particle(g, np, p, xi, u, E, B, J, q, m, w);
}

/* ----------------------------------------------------------------------- */
/* FDTD (discrete curls nabla^+ x E and nabla^- x B, leap-frog)             */
/* ----------------------------------------------------------------------- */

/* B <- B - h * curl^+ E  (h = dt/2 for the half steps of fig. psc_new) */
void orc_push_b(const orc_grid *g, const double *E, double *B, double h) {
    long nc = ncell(g);
    const double *Ex = E, *Ey = E + nc, *Ez = E + 2 * nc;
    double *Bx = B, *By = B + nc, *Bz = B + 2 * nc;
    double ix = active(g, 0) ? 1.0 / g->d[0] : 0.0, iy = 1.0 / g->d[1], iz = 1.0 / g->d[2];
#pragma omp parallel for
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long c = idx3(g, i, j, k);
                double cx = (Ez[idx3(g, i, j + 1, k)] - Ez[c]) * iy - (Ey[idx3(g, i, j, k + 1)] - Ey[c]) * iz;
                double cy = (Ex[idx3(g, i, j, k + 1)] - Ex[c]) * iz - (Ez[idx3(g, i + 1, j, k)] - Ez[c]) * ix;
                double cz = (Ey[idx3(g, i + 1, j, k)] - Ey[c]) * ix - (Ex[idx3(g, i, j + 1, k)] - Ex[c]) * iy;
                Bx[c] -= h * cx;
                By[c] -= h * cy;
                Bz[c] -= h * cz;
            }
}

/* E <- E + dt * (curl^- B - J) */
void orc_push_e(const orc_grid *g, double *E, const double *B, const double *J, double h) {
    long nc = ncell(g);
    double *Ex = E, *Ey = E + nc, *Ez = E + 2 * nc;
    const double *Bx = B, *By = B + nc, *Bz = B + 2 * nc;
    const double *Jx = J, *Jy = J + nc, *Jz = J + 2 * nc;
    double ix = active(g, 0) ? 1.0 / g->d[0] : 0.0, iy = 1.0 / g->d[1], iz = 1.0 / g->d[2];
#pragma omp parallel for
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long c = idx3(g, i, j, k);
                double cx = (Bz[c] - Bz[idx3(g, i, j - 1, k)]) * iy - (By[c] - By[idx3(g, i, j, k - 1)]) * iz;
                double cy = (Bx[c] - Bx[idx3(g, i, j, k - 1)]) * iz - (Bz[c] - Bz[idx3(g, i - 1, j, k)]) * ix;
                double cz = (By[c] - By[idx3(g, i - 1, j, k)]) * ix - (Bx[c] - Bx[idx3(g, i, j - 1, k)]) * iy;
                Ex[c] += h * (cx - (J ? Jx[c] : 0.0));
                Ey[c] += h * (cy - (J ? Jy[c] : 0.0));
                Ez[c] += h * (cz - (J ? Jz[c] : 0.0));
            }
}

/* nabla^- . E at nodes */
void orc_div_e(const orc_grid *g, const double *E, double *out) {
    long nc = ncell(g);
    double ix = active(g, 0) ? 1.0 / g->d[0] : 0.0, iy = 1.0 / g->d[1], iz = 1.0 / g->d[2];
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long c = idx3(g, i, j, k);
                out[c] = (E[c] - E[idx3(g, i - 1, j, k)]) * ix +
                         (E[nc + c] - E[nc + idx3(g, i, j - 1, k)]) * iy +
                         (E[2 * nc + c] - E[2 * nc + idx3(g, i, j, k - 1)]) * iz;
            }
}

/* Marder's divergence cleaning (the iterative method the paper names for
 * dissipating violations of Gauss's law): E += d dt nabla^+ F for a field F
 * at nodes, F being the Gauss residual nabla^- . E - rho (less a reference).
 * The forward difference of a node quantity sits where E is staggered. */
void orc_marder(const orc_grid *g, double *E, const double *F, double d) {
    long nc = ncell(g);
    double ix = active(g, 0) ? 1.0 / g->d[0] : 0.0, iy = 1.0 / g->d[1], iz = 1.0 / g->d[2];
    double h = d * g->dt;
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long c = idx3(g, i, j, k);
                E[c] += h * (F[idx3(g, i + 1, j, k)] - F[c]) * ix;
                E[nc + c] += h * (F[idx3(g, i, j + 1, k)] - F[c]) * iy;
                E[2 * nc + c] += h * (F[idx3(g, i, j, k + 1)] - F[c]) * iz;
            }
}

/* nabla^+ . B at cell centres */
void orc_div_b(const orc_grid *g, const double *B, double *out) {
    long nc = ncell(g);
    double ix = active(g, 0) ? 1.0 / g->d[0] : 0.0, iy = 1.0 / g->d[1], iz = 1.0 / g->d[2];
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long c = idx3(g, i, j, k);
                out[c] = (B[idx3(g, i + 1, j, k)] - B[c]) * ix +
                         (B[nc + idx3(g, i, j + 1, k)] - B[nc + c]) * iy +
                         (B[2 * nc + idx3(g, i, j, k + 1)] - B[2 * nc + c]) * iz;
            }
}

/* Charge density at nodes: rho(node) += q w prod_d b(xi_d - node_d) */
void orc_deposit_rho(const orc_grid *g, long np, const double *xi, double qw, double *rho) {
    for (long p = 0; p < np; ++p) {
        double x[3];
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            x[d] = xi[d * np + p];
            if (!active(g, d)) continue;
            lo[d] = (int)floor(x[d]) - 2;
            hi[d] = lo[d] + 5;
        }
        for (int k = lo[2]; k <= hi[2]; ++k) {
            double wz = active(g, 2) ? orc_bspline(g->order, x[2] - k) : 1.0;
            for (int j = lo[1]; j <= hi[1]; ++j) {
                double wy = active(g, 1) ? orc_bspline(g->order, x[1] - j) : 1.0;
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    double wx = active(g, 0) ? orc_bspline(g->order, x[0] - i) : 1.0;
                    double s = wx * wy * wz;
                    if (s != 0.0) rho[idx3(g, i, j, k)] += qw * s;
                }
            }
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Sort (sec. "Sorting and Communication")                                 */
/* ----------------------------------------------------------------------- */

/* Patch-major cell key: patches tile the grid in row-major patch order (x
 * fastest), edge patches truncated; cells inside a patch row-major.  The
 * key of a cell is its rank in that enumeration, built here by plain
 * enumeration.  key_of_cell has ncell entries, indexed by geometric index. */
void orc_patch_keys(const orc_grid *g, const int patch[3], int32_t *key_of_cell) {
    int np[3];
    for (int d = 0; d < 3; ++d) np[d] = (g->n[d] + patch[d] - 1) / patch[d];
    int32_t next = 0;
    for (int pk = 0; pk < np[2]; ++pk)
        for (int pj = 0; pj < np[1]; ++pj)
            for (int pi = 0; pi < np[0]; ++pi) {
                int o[3] = {pi * patch[0], pj * patch[1], pk * patch[2]};
                int e[3];
                for (int d = 0; d < 3; ++d) e[d] = (o[d] + patch[d] < g->n[d]) ? o[d] + patch[d] : g->n[d];
                for (int k = o[2]; k < e[2]; ++k)
                    for (int j = o[1]; j < e[1]; ++j)
                        for (int i = o[0]; i < e[0]; ++i)
                            key_of_cell[idx3(g, i, j, k)] = next++;
            }
}

/* Stable counting sort: perm[r] = index of the r-th particle in key order,
 * equal keys in their input order.  Returns 0, or -1 if a key is out of range. */
int orc_stable_sort(long n, const int32_t *keys, int32_t nkeys, int32_t *perm) {
    long *start = (long *)calloc((size_t)nkeys + 1, sizeof(long));
    if (!start) return -1;
    for (long p = 0; p < n; ++p) {
        if (keys[p] < 0 || keys[p] >= nkeys) { free(start); return -1; }
        start[keys[p] + 1]++;
    }
    for (int32_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];
    for (long p = 0; p < n; ++p) perm[start[keys[p]]++] = (int32_t)p;
    free(start);
    return 0;
}

/* Geometric cell of an absolute position (floor per active dimension). */
long orc_cell_of(const orc_grid *g, const double x[3]) {
    int c[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d)
        if (active(g, d)) c[d] = wrapi((int)floor(x[d]), g->n[d]);
    return idx3(g, c[0], c[1], c[2]);
}

/* ----------------------------------------------------------------------- */
/* Diagnostics                                                             */
/* ----------------------------------------------------------------------- */

/* 0.5 * sum(F^2) * dV over one 3-component field */
double orc_field_energy(const orc_grid *g, const double *F) {
    long nc = ncell(g);
    double dV = g->d[1] * g->d[2] * (g->dim == 3 ? g->d[0] : 1.0);
    double s = 0.0;
    for (long c = 0; c < 3 * nc; ++c) s += F[c] * F[c];
    return 0.5 * s * dV;
}

/* sum m w dV (gamma - 1) */
double orc_kinetic_energy(const orc_grid *g, long np, const double *u, double m, double w) {
    double dV = g->d[1] * g->d[2] * (g->dim == 3 ? g->d[0] : 1.0);
    double s = 0.0;
    for (long p = 0; p < np; ++p) {
        double u2 = u[p] * u[p] + u[np + p] * u[np + p] + u[2 * np + p] * u[2 * np + p];
        s += sqrt(1.0 + u2) - 1.0;
    }
    return m * w * dV * s;
}
