/* Drives every routine of the double-precision oracle on small 2-d and 3-d
 * runs (orders 1 and 2, Esirkepov and Villasenor-Buneman deposits, particles
 * on cell faces and at the grid edges, several whole steps) so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer sees every memory
 * access and integer operation of the oracle.  Compiled and run by
 * tests/test_oracle_sanitized.py; exits non-zero if a result is not finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int dim, n[3];
    double d[3], dt;
    int order, vb;
} orc_grid;

double orc_bspline(int order, double s);
double orc_interp(const orc_grid *g, const double *F, const double xi[3], const double stag[3]);
void orc_boris(double u[3], const double E[3], const double B[3], double qdt_2m);
void orc_deposit(const orc_grid *g, double *J, const double xi0[3], const double xi1[3], double qw, double vx);
void orc_deposit_vb(const orc_grid *g, double *J, const double xi0[3], const double xi1[3], double qw, double vx);
void orc_push_particles(const orc_grid *g, long np, double *xi, double *u, const double *E, const double *B,
                        double *J, double q, double m, double w);
void orc_push_b(const orc_grid *g, const double *E, double *B, double h);
void orc_push_e(const orc_grid *g, double *E, const double *B, const double *J, double h);
void orc_div_e(const orc_grid *g, const double *E, double *out);
void orc_marder(const orc_grid *g, double *E, const double *F, double d);
void orc_div_b(const orc_grid *g, const double *B, double *out);
void orc_deposit_rho(const orc_grid *g, long np, const double *xi, double qw, double *rho);
void orc_patch_keys(const orc_grid *g, const int patch[3], int32_t *key_of_cell);
int orc_stable_sort(long n, const int32_t *keys, int32_t nkeys, int32_t *perm);
long orc_cell_of(const orc_grid *g, const double x[3]);
double orc_field_energy(const orc_grid *g, const double *F);
double orc_kinetic_energy(const orc_grid *g, long np, const double *u, double m, double w);

/* splitmix64: seeded test inputs only */
static uint64_t state = 1310;
static double uniform(void) {
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int check(const char *what, const double *a, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) {
            printf("%s: non-finite value at %ld\n", what, i);
            return 1;
        }
    return 0;
}

static int run(int dim, int order, int vb, int nx, int ny, int nz, const int patch[3]) {
    orc_grid g = {dim, {dim == 3 ? nx : 1, ny, nz}, {0.1, 0.1, 0.1}, 0.0, order, vb};
    double s = 0.0;
    for (int d = 0; d < 3; ++d)
        if (dim == 3 || d > 0) s += 1.0 / (g.d[d] * g.d[d]);
    g.dt = 0.5 / sqrt(s);
    const long nc = (long)g.n[0] * g.n[1] * g.n[2];
    const long np = 8 * nc;
    double *E = calloc(3 * nc, sizeof(double)), *B = calloc(3 * nc, sizeof(double));
    double *J = calloc(3 * nc, sizeof(double)), *rho = calloc(nc, sizeof(double));
    double *div = calloc(nc, sizeof(double)), *xi = malloc(3 * np * sizeof(double));
    double *u = malloc(3 * np * sizeof(double));
    int32_t *key_of_cell = malloc(nc * sizeof(int32_t)), *keys = malloc(np * sizeof(int32_t));
    int32_t *perm = malloc(np * sizeof(int32_t));
    int bad = 0;
    for (long i = 0; i < 3 * nc; ++i) {
        E[i] = 0.05 * (uniform() - 0.5);
        B[i] = 0.3 * (uniform() - 0.5);
    }
    for (long p = 0; p < np; ++p)
        for (int d = 0; d < 3; ++d) {
            double x = (dim == 3 || d > 0) ? uniform() * g.n[d] : 0.0;
            if (p % 17 == 0 && (dim == 3 || d > 0)) x = floor(x);              /* on a cell face */
            if (p % 29 == 0 && (dim == 3 || d > 0)) x = g.n[d] - 1e-12;         /* at the upper edge */
            xi[d * np + p] = x;
            u[d * np + p] = 0.4 * (uniform() - 0.5);
        }
    for (int step = 0; step < 4; ++step) {
        orc_push_b(&g, E, B, 0.5 * g.dt);
        for (long i = 0; i < 3 * nc; ++i) J[i] = 0.0;
        orc_push_particles(&g, np, xi, u, E, B, J, -1.0, 1.0, 0.125);
        orc_push_b(&g, E, B, 0.5 * g.dt);
        orc_push_e(&g, E, B, J, g.dt);
        orc_patch_keys(&g, patch, key_of_cell);
        for (long p = 0; p < np; ++p) {
            const double x[3] = {xi[p], xi[np + p], xi[2 * np + p]};
            keys[p] = key_of_cell[orc_cell_of(&g, x)];
        }
        if (orc_stable_sort(np, keys, (int32_t)nc, perm) != 0) bad = 1;
    }
    for (long i = 0; i < nc; ++i) rho[i] = 0.0;
    orc_deposit_rho(&g, np, xi, -0.125, rho);
    orc_div_e(&g, E, div);
    for (long i = 0; i < nc; ++i) div[i] -= rho[i];
    orc_marder(&g, E, div, 0.1 * g.dt);
    orc_div_b(&g, B, div);
    /* single-particle entry points, including a cell-crossing move */
    {
        double x0[3] = {dim == 3 ? 1.95 : 0.0, 2.95, 1.02}, x1[3] = {dim == 3 ? 2.05 : 0.0, 3.03, 0.97};
        double uu[3] = {0.1, -0.2, 0.3}, Ep[3] = {0.01, 0.02, -0.01}, Bp[3] = {0.1, 0.0, 0.2};
        const double stag[3] = {0.5, 0.0, 0.5};
        orc_deposit(&g, J, x0, x1, 0.125, 0.1);
        orc_deposit_vb(&g, J, x0, x1, 0.125, 0.1);
        orc_boris(uu, Ep, Bp, 0.01);
        double v = orc_interp(&g, E, x0, stag) + orc_bspline(order, 0.3) + orc_bspline(order, 1.2);
        if (!isfinite(v)) bad = 1;
    }
    double w = orc_field_energy(&g, E) + orc_field_energy(&g, B) + orc_kinetic_energy(&g, np, u, 1.0, 0.125);
    bad |= check("E", E, 3 * nc) | check("B", B, 3 * nc) | check("J", J, 3 * nc) | check("xi", xi, 3 * np) |
           !isfinite(w);
    printf("dim %d order %d vb %d grid %dx%dx%d: energy %.6e\n", dim, order, vb, g.n[0], g.n[1], g.n[2], w);
    free(E); free(B); free(J); free(rho); free(div); free(xi); free(u); free(key_of_cell); free(keys); free(perm);
    return bad;
}

int main(void) {
    const int p2[3] = {1, 4, 3}, p3[3] = {3, 4, 2};
    int bad = 0;
    for (int order = 1; order <= 2; ++order) {
        bad |= run(2, order, 0, 1, 10, 7, p2);
        bad |= run(3, order, 0, 7, 6, 5, p3);
    }
    bad |= run(2, 1, 1, 1, 9, 8, p2);
    bad |= run(3, 1, 1, 5, 6, 7, p3);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
