/*
 * sanitize_driver.c -- test infrastructure: runs every entry point of the two
 * oracles on tiny and degenerate lattices so that a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer can check their indexing (the test suite
 * builds and runs it; nothing else uses it).  Exit status 0 when every call
 * returned success and the Tau1 and LBGK forms agreed.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* entry points of tau1_oracle.c and tau1_oracle_2d.c (linked in) */
int tau1o_run(int q, long nx, long ny, long nz, const uint8_t *solid, double *drho, double *ux,
              double *uy, double *uz, const double *g, long nsteps, int nthreads);
int tau1o_step_nodes(int q, long nx, long ny, long nz, const uint8_t *solid, const double *drho,
                     const double *ux, const double *uy, const double *uz, const double *g,
                     long nidx, const long *idx, double *out, int nthreads);
int tau1o_run_rhoform(int q, long nx, long ny, long nz, const uint8_t *solid, double *rho,
                      double *ux, double *uy, double *uz, const double *g, long nsteps,
                      int nthreads);
int tau1o_bgk_run(int q, long nx, long ny, long nz, const uint8_t *solid, double *drho,
                  double *ux, double *uy, double *uz, const double *g, double omega, long nsteps,
                  int nthreads);
int tau1o_reduce(long nx, long ny, long nz, const uint8_t *solid, const double *drho,
                 const double *ux, const double *uy, const double *uz, int axis, double g_axis,
                 double *mass, double *perm);
int tau1o2_run(long nx, long ny, const uint8_t *type, double *drho, double *ux, double *uy,
               const double *g, const double *uw, int xbc, double rho_in, double rho_out,
               long nsteps, int nthreads);
int tau1o2_bgk_run(long nx, long ny, const uint8_t *type, double *drho, double *ux, double *uy,
                   const double *g, const double *uw, int xbc, double rho_in, double rho_out,
                   double omega, long nsteps);
int tau1o2_reduce(long nx, long ny, const uint8_t *type, const double *drho, const double *ux,
                  double *mass, double *mean_ux);

static unsigned long rng = 12345;
static double urand(void)
{
    rng = rng * 6364136223846793005UL + 1442695040888963407UL;
    return (double)(rng >> 11) / 9007199254740992.0;
}

static int case3(int q, long nx, long ny, long nz)
{
    const long n = nx * ny * nz;
    uint8_t *solid = malloc((size_t)n);
    double *a = calloc((size_t)(8 * n), sizeof(double));
    double *out = calloc((size_t)(4 * n), sizeof(double));
    long *idx = malloc(sizeof(long) * (size_t)n);
    double g[3] = {1e-5, -2e-5, 3e-6}, m, k;
    long i;
    int rc = 0;
    for (i = 0; i < n; ++i) {
        solid[i] = urand() < 0.3;
        a[i] = solid[i] ? 0.0 : 1e-3 * (urand() - 0.5);
        a[n + i] = solid[i] ? 0.0 : 0.05 * (urand() - 0.5);
        a[2 * n + i] = solid[i] ? 0.0 : 0.05 * (urand() - 0.5);
        a[3 * n + i] = solid[i] ? 0.0 : 0.05 * (urand() - 0.5);
        idx[i] = i;
    }
    memcpy(a + 4 * n, a, sizeof(double) * 4 * (size_t)n);
    rc |= tau1o_step_nodes(q, nx, ny, nz, solid, a, a + n, a + 2 * n, a + 3 * n, g, n, idx, out, 1);
    rc |= tau1o_run(q, nx, ny, nz, solid, a, a + n, a + 2 * n, a + 3 * n, g, 3, 1);
    rc |= tau1o_bgk_run(q, nx, ny, nz, solid, a + 4 * n, a + 5 * n, a + 6 * n, a + 7 * n, g, 1.0, 3, 1);
    for (i = 0; i < 4 * n; ++i)
        if (a[i] != a[4 * n + i]) rc |= 2;
    rc |= tau1o_reduce(nx, ny, nz, solid, a, a + n, a + 2 * n, a + 3 * n, 0, g[0], &m, &k);
    for (i = 0; i < n; ++i) a[i] += 1.0;
    rc |= tau1o_run_rhoform(q, nx, ny, nz, solid, a, a + n, a + 2 * n, a + 3 * n, g, 2, 1);
    free(solid);
    free(a);
    free(out);
    free(idx);
    if (rc) fprintf(stderr, "3-D case q=%d %ldx%ldx%ld failed (%d)\n", q, nx, ny, nz, rc);
    return rc;
}

static int case2(long nx, long ny, int xbc)
{
    const long n = nx * ny;
    uint8_t *t = malloc((size_t)n);
    double *a = calloc((size_t)(6 * n), sizeof(double));
    double g[2] = {1e-5, 0.0}, uw[2] = {0.05, 0.0}, m, s;
    long i;
    int rc = 0;
    for (i = 0; i < n; ++i) {
        t[i] = urand() < 0.15 ? (urand() < 0.5 ? 1 : 2) : 0;
        a[i] = t[i] ? 0.0 : 1e-3 * (urand() - 0.5);
        a[n + i] = t[i] ? 0.0 : 0.05 * (urand() - 0.5);
        a[2 * n + i] = t[i] ? 0.0 : 0.05 * (urand() - 0.5);
    }
    memcpy(a + 3 * n, a, sizeof(double) * 3 * (size_t)n);
    rc |= tau1o2_run(nx, ny, t, a, a + n, a + 2 * n, g, uw, xbc, 1.01, 0.99, 4, 1);
    rc |= tau1o2_bgk_run(nx, ny, t, a + 3 * n, a + 4 * n, a + 5 * n, g, uw, xbc, 1.01, 0.99, 1.0, 4);
    for (i = 0; i < 3 * n; ++i)
        if (fabs(a[i] - a[3 * n + i]) > 1e-15) rc |= 2;
    rc |= tau1o2_reduce(nx, ny, t, a, a + n, &m, &s);
    free(t);
    free(a);
    if (rc) fprintf(stderr, "2-D case %ldx%ld xbc=%d failed (%d)\n", nx, ny, xbc, rc);
    return rc;
}

int main(void)
{
    static const long dims[][3] = {{1, 1, 1}, {2, 1, 1}, {1, 3, 1}, {1, 1, 4}, {5, 3, 7}, {4, 6, 2}};
    static const int qs[] = {15, 19, 27};
    static const long d2[][2] = {{1, 1}, {3, 1}, {1, 5}, {7, 4}, {12, 9}};
    int rc = 0;
    unsigned a, b;
    for (a = 0; a < sizeof qs / sizeof qs[0]; ++a)
        for (b = 0; b < sizeof dims / sizeof dims[0]; ++b)
            rc |= case3(qs[a], dims[b][0], dims[b][1], dims[b][2]);
    for (b = 0; b < sizeof d2 / sizeof d2[0]; ++b) {
        rc |= case2(d2[b][0], d2[b][1], 0);
        if (d2[b][0] >= 3) rc |= case2(d2[b][0], d2[b][1], 1);
    }
    printf(rc ? "FAILED\n" : "ok\n");
    return rc ? 1 : 0;
}
