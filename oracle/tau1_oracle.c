/*
 * tau1_oracle.c -- plain, slow, FP64 CPU oracle for the Tau1 lattice
 * Boltzmann update (relaxation time equal to one).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the GPU path.
 *
 * What it computes (Bacza, Tomczak, Matyka, "The lattice Boltzmann method for
 * fluid flows at relaxation time equal one: performance study"):
 *
 *   * Eq. (4) with tau = 1 reduces to Eq. (8): the population that arrives at
 *     x along c_k at t+1 is the equilibrium of Eq. (3) evaluated at the
 *     source node x - c_k at time t.  Only rho and u are stored (algorithm
 *     "Tau1" of the AB-layout comparison figure, pull form).
 *   * Eqs. (9)-(10): the new density and momentum are the zeroth and first
 *     moments of those arriving equilibria (Eq. (10) read as the momentum
 *     j, divided by rho afterwards, as in the division-saving algorithm of
 *     the implementation section: one reciprocal per node).
 *   * Halfway bounce-back (Eq. (11) and the bounce-back algorithm of the
 *     wall-boundary subsection): when the source x - c_k is a wall, the
 *     missing population is rebuilt from the node's own previous rho*, u*
 *     with the opposite direction; it is still counted as arriving along c_k.
 *   * Periodic wrap on every axis; walls are solid nodes.
 *   * Body force (not in the paper): velocity-shift form, the equilibrium is
 *     evaluated at v = u + g/2 and the stored physical velocity is
 *     u = j/rho + g/2, g an acceleration in lattice units.
 *
 * The state is held as (drho = rho - 1, u).  The arriving value is stored
 * minus its weight, f' = f_eq - w_k = w_k (drho_s + rho_s P), which keeps the
 * O(1) part out of the sums; the dropped weights add up to exactly 1 and
 * exactly 0 in the first moment, so nothing is lost.
 *
 * Also here:
 *   * tau1o_bgk_run: a brute-force standard LBGK with full populations, pull
 *     streaming and the same bounce-back (the "Standard LBM" algorithm of the
 *     comparison figure, collision (1-omega) f + omega f_eq).  At omega = 1 it
 *     must reproduce tau1o_run exactly.
 *   * tau1o_run_rhoform: the same method written with rho instead of drho,
 *     Eq. (3) as printed; agrees with the drho form to rounding.
 *   * tau1o_step_nodes: one update at selected nodes only.
 *   * tau1o_reduce: mass and Darcy permeability of a state.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (never fast-math).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 27

typedef struct {
    int q;
    int c[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
} lattice_t;

/* Direction order: rest; the six faces +x -x +y -y +z -z; the twelve edges
 * as six opposite pairs; the eight corners as four opposite pairs.  Each
 * non-rest direction is followed by its opposite, so opp(k) = k + 1 for odd k
 * and k - 1 for even k >= 2. */
static const int FACE[6][3] = {
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const int EDGE[12][3] = {
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const int CORNER[8][3] = {
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

/* Textbook weights of the DdQq sets (Qian, d'Humieres, Lallemand 1992); the
 * paper names the sets but does not list them. */
static int make_lattice(int q, lattice_t *L)
{
    double w0, wf, we, wc;
    int use_edges, use_corners, k = 0, i;
    if (q == 15) {
        w0 = 2.0 / 9.0; wf = 1.0 / 9.0; we = 0.0; wc = 1.0 / 72.0;
        use_edges = 0; use_corners = 1;
    } else if (q == 19) {
        w0 = 1.0 / 3.0; wf = 1.0 / 18.0; we = 1.0 / 36.0; wc = 0.0;
        use_edges = 1; use_corners = 0;
    } else if (q == 27) {
        w0 = 8.0 / 27.0; wf = 2.0 / 27.0; we = 1.0 / 54.0; wc = 1.0 / 216.0;
        use_edges = 1; use_corners = 1;
    } else {
        return -1;
    }
    L->q = q;
    L->c[k][0] = L->c[k][1] = L->c[k][2] = 0;
    L->w[k++] = w0;
    for (i = 0; i < 6; ++i, ++k) {
        memcpy(L->c[k], FACE[i], sizeof FACE[i]);
        L->w[k] = wf;
    }
    if (use_edges)
        for (i = 0; i < 12; ++i, ++k) {
            memcpy(L->c[k], EDGE[i], sizeof EDGE[i]);
            L->w[k] = we;
        }
    if (use_corners)
        for (i = 0; i < 8; ++i, ++k) {
            memcpy(L->c[k], CORNER[i], sizeof CORNER[i]);
            L->w[k] = wc;
        }
    L->opp[0] = 0;
    for (i = 1; i < q; ++i) L->opp[i] = (i % 2 == 1) ? i + 1 : i - 1;
    return 0;
}

int tau1o_lattice(int q, int *c, double *w, int *opp)
{
    lattice_t L;
    int k;
    if (make_lattice(q, &L)) return -1;
    for (k = 0; k < q; ++k) {
        c[3 * k + 0] = L.c[k][0];
        c[3 * k + 1] = L.c[k][1];
        c[3 * k + 2] = L.c[k][2];
        w[k] = L.w[k];
        opp[k] = L.opp[k];
    }
    return q;
}

static long wrap(long a, long n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* Eq. (3) with c_s^2 = 1/3, minus its weight, at density 1 + ds and velocity
 * v, for direction cd and weight wk. */
static double feq_minus_w(double wk, const int *cd, double ds, double vx,
                          double vy, double vz)
{
    double rho = 1.0 + ds;
    double cu = ((double)cd[0] * vx + (double)cd[1] * vy) + (double)cd[2] * vz;
    double vv = (vx * vx + vy * vy) + vz * vz;
    double p = (3.0 * cu + (4.5 * cu) * cu) - 1.5 * vv;
    return wk * (ds + rho * p);
}

typedef struct {
    long nx, ny, nz;
    const uint8_t *solid;
    double gh[3];
} grid_t;

/* One Tau1 update of fluid node (x, y, z) reading the pre-step state;
 * writes drho', u' into out[0..3]. */
static void tau1_node(const lattice_t *L, const grid_t *G, long x, long y,
                      long z, const double *dr, const double *ux,
                      const double *uy, const double *uz, double out[4])
{
    const long nx = G->nx, ny = G->ny, nz = G->nz;
    const long i = x + nx * (y + ny * z);
    double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, r;
    int k;
    for (k = 0; k < L->q; ++k) {
        long sx = wrap(x - L->c[k][0], nx);
        long sy = wrap(y - L->c[k][1], ny);
        long sz = wrap(z - L->c[k][2], nz);
        long s = sx + nx * (sy + ny * sz);
        long src;
        int dir;
        double f;
        if (!G->solid[s]) {
            src = s;
            dir = k;
        } else {
            /* halfway bounce-back: own previous state, opposite direction */
            src = i;
            dir = L->opp[k];
        }
        f = feq_minus_w(L->w[k], L->c[dir], dr[src], ux[src] + G->gh[0],
                        uy[src] + G->gh[1], uz[src] + G->gh[2]);
        d += f;
        jx += (double)L->c[k][0] * f;
        jy += (double)L->c[k][1] * f;
        jz += (double)L->c[k][2] * f;
    }
    r = 1.0 / (1.0 + d);
    out[0] = d;
    out[1] = jx * r + G->gh[0];
    out[2] = jy * r + G->gh[1];
    out[3] = jz * r + G->gh[2];
}

static int check_args(long nx, long ny, long nz, const uint8_t *solid)
{
    if (nx < 1 || ny < 1 || nz < 1 || !solid) return -1;
    return 0;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int tau1o_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Advance (drho, u) in place by nsteps Tau1 updates.  Solid nodes are never
 * read as sources and are reported as drho = 0, u = 0. */
int tau1o_run(int q, long nx, long ny, long nz, const uint8_t *solid,
              double *drho, double *ux, double *uy, double *uz,
              const double *g, long nsteps, int nthreads)
{
    lattice_t L;
    grid_t G;
    long N, n, i;
    double *buf, *pre[4], *post[4];
    if (make_lattice(q, &L) || check_args(nx, ny, nz, solid) || nsteps < 0)
        return -1;
    set_threads(nthreads);
    N = nx * ny * nz;
    G.nx = nx; G.ny = ny; G.nz = nz; G.solid = solid;
    G.gh[0] = 0.5 * g[0]; G.gh[1] = 0.5 * g[1]; G.gh[2] = 0.5 * g[2];
    buf = (double *)malloc(sizeof(double) * 4 * (size_t)N);
    if (!buf) return -2;
    pre[0] = drho; pre[1] = ux; pre[2] = uy; pre[3] = uz;
    for (i = 0; i < 4; ++i) post[i] = buf + i * N;
    for (i = 0; i < N; ++i)
        if (solid[i]) drho[i] = ux[i] = uy[i] = uz[i] = 0.0;
    for (i = 0; i < 4; ++i) memcpy(post[i], pre[i], sizeof(double) * (size_t)N);

    for (n = 0; n < nsteps; ++n) {
        long z;
#pragma omp parallel for schedule(static)
        for (z = 0; z < nz; ++z) {
            long y, x;
            double out[4];
            for (y = 0; y < ny; ++y)
                for (x = 0; x < nx; ++x) {
                    long j = x + nx * (y + ny * z);
                    if (solid[j]) continue;
                    tau1_node(&L, &G, x, y, z, pre[0], pre[1], pre[2], pre[3],
                              out);
                    post[0][j] = out[0];
                    post[1][j] = out[1];
                    post[2][j] = out[2];
                    post[3][j] = out[3];
                }
        }
        for (i = 0; i < 4; ++i) {
            double *t = pre[i];
            pre[i] = post[i];
            post[i] = t;
        }
    }
    /* the caller's arrays hold the result */
    if (pre[0] != drho) {
        memcpy(drho, pre[0], sizeof(double) * (size_t)N);
        memcpy(ux, pre[1], sizeof(double) * (size_t)N);
        memcpy(uy, pre[2], sizeof(double) * (size_t)N);
        memcpy(uz, pre[3], sizeof(double) * (size_t)N);
    }
    free(buf);
    return 0;
}

/* One update at the listed node indices (x + nx*(y + ny*z)) from a full
 * pre-step state; out holds 4 values per listed node (drho', ux', uy', uz'),
 * zeros for solid nodes. */
int tau1o_step_nodes(int q, long nx, long ny, long nz, const uint8_t *solid,
                     const double *drho, const double *ux, const double *uy,
                     const double *uz, const double *g, long nidx,
                     const long *idx, double *out, int nthreads)
{
    lattice_t L;
    grid_t G;
    long m;
    if (make_lattice(q, &L) || check_args(nx, ny, nz, solid) || nidx < 0)
        return -1;
    set_threads(nthreads);
    G.nx = nx; G.ny = ny; G.nz = nz; G.solid = solid;
    G.gh[0] = 0.5 * g[0]; G.gh[1] = 0.5 * g[1]; G.gh[2] = 0.5 * g[2];
    for (m = 0; m < nidx; ++m)
        if (idx[m] < 0 || idx[m] >= nx * ny * nz) return -1;
#pragma omp parallel for schedule(static)
    for (m = 0; m < nidx; ++m) {
        long j = idx[m];
        long x = j % nx, y = (j / nx) % ny, z = j / (nx * ny);
        if (solid[j]) {
            out[4 * m + 0] = out[4 * m + 1] = out[4 * m + 2] =
                out[4 * m + 3] = 0.0;
        } else {
            tau1_node(&L, &G, x, y, z, drho, ux, uy, uz, out + 4 * m);
        }
    }
    return 0;
}

/* The same update with the state held as rho (not rho - 1) and the
 * equilibrium of Eq. (3) evaluated as printed:
 *   f = w rho_s (1 + 3 cu + 4.5 cu^2 - 1.5 v.v).
 * rho is in/out (physical density), u in/out. */
int tau1o_run_rhoform(int q, long nx, long ny, long nz, const uint8_t *solid,
                      double *rho, double *ux, double *uy, double *uz,
                      const double *g, long nsteps, int nthreads)
{
    lattice_t L;
    long N, n, i;
    double gh[3], *buf, *pre[4], *post[4];
    if (make_lattice(q, &L) || check_args(nx, ny, nz, solid) || nsteps < 0)
        return -1;
    set_threads(nthreads);
    N = nx * ny * nz;
    gh[0] = 0.5 * g[0]; gh[1] = 0.5 * g[1]; gh[2] = 0.5 * g[2];
    buf = (double *)malloc(sizeof(double) * 4 * (size_t)N);
    if (!buf) return -2;
    pre[0] = rho; pre[1] = ux; pre[2] = uy; pre[3] = uz;
    for (i = 0; i < 4; ++i) post[i] = buf + i * N;
    for (i = 0; i < N; ++i)
        if (solid[i]) { rho[i] = 1.0; ux[i] = uy[i] = uz[i] = 0.0; }
    for (i = 0; i < 4; ++i) memcpy(post[i], pre[i], sizeof(double) * (size_t)N);

    for (n = 0; n < nsteps; ++n) {
        long z;
#pragma omp parallel for schedule(static)
        for (z = 0; z < nz; ++z) {
            long y, x;
            for (y = 0; y < ny; ++y)
                for (x = 0; x < nx; ++x) {
                    long j = x + nx * (y + ny * z);
                    double rs = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, r;
                    int k;
                    if (solid[j]) continue;
                    for (k = 0; k < q; ++k) {
                        long sx = wrap(x - L.c[k][0], nx);
                        long sy = wrap(y - L.c[k][1], ny);
                        long sz = wrap(z - L.c[k][2], nz);
                        long s = sx + nx * (sy + ny * sz), src = s;
                        int dir = k;
                        double vx, vy, vz, cu, vv, f;
                        if (solid[s]) { src = j; dir = L.opp[k]; }
                        vx = pre[1][src] + gh[0];
                        vy = pre[2][src] + gh[1];
                        vz = pre[3][src] + gh[2];
                        cu = ((double)L.c[dir][0] * vx + (double)L.c[dir][1] * vy)
                             + (double)L.c[dir][2] * vz;
                        vv = (vx * vx + vy * vy) + vz * vz;
                        f = L.w[k] * pre[0][src]
                            * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * vv);
                        rs += f;
                        jx += (double)L.c[k][0] * f;
                        jy += (double)L.c[k][1] * f;
                        jz += (double)L.c[k][2] * f;
                    }
                    r = 1.0 / rs;
                    post[0][j] = rs;
                    post[1][j] = jx * r + gh[0];
                    post[2][j] = jy * r + gh[1];
                    post[3][j] = jz * r + gh[2];
                }
        }
        for (i = 0; i < 4; ++i) {
            double *t = pre[i];
            pre[i] = post[i];
            post[i] = t;
        }
    }
    if (pre[0] != rho) {
        memcpy(rho, pre[0], sizeof(double) * (size_t)N);
        memcpy(ux, pre[1], sizeof(double) * (size_t)N);
        memcpy(uy, pre[2], sizeof(double) * (size_t)N);
        memcpy(uz, pre[3], sizeof(double) * (size_t)N);
    }
    free(buf);
    return 0;
}

/* Brute-force standard LBGK (Eq. (4)) with full populations, pull streaming
 * over two copies (AB layout) and halfway bounce-back at solid links.
 * Populations are held minus their weights (f' = f - w_k).  Collision:
 * f'post = (1 - omega) f' + omega f'eq(drho, u + g/2); moments in direction
 * order, u = j / (1 + drho) + g/2.  The state (drho, u) is in/out, as in
 * tau1o_run; the populations start at equilibrium of that state. */
int tau1o_bgk_run(int q, long nx, long ny, long nz, const uint8_t *solid,
                  double *drho, double *ux, double *uy, double *uz,
                  const double *g, double omega, long nsteps, int nthreads)
{
    lattice_t L;
    long N, n, i;
    double gh[3], *fa, *fb;
    if (make_lattice(q, &L) || check_args(nx, ny, nz, solid) || nsteps < 0)
        return -1;
    set_threads(nthreads);
    N = nx * ny * nz;
    gh[0] = 0.5 * g[0]; gh[1] = 0.5 * g[1]; gh[2] = 0.5 * g[2];
    fa = (double *)malloc(sizeof(double) * (size_t)q * (size_t)N);
    fb = (double *)malloc(sizeof(double) * (size_t)q * (size_t)N);
    if (!fa || !fb) { free(fa); free(fb); return -2; }
    for (i = 0; i < N; ++i) {
        int k;
        if (solid[i]) {
            drho[i] = ux[i] = uy[i] = uz[i] = 0.0;
            for (k = 0; k < q; ++k) fa[(size_t)k * N + i] = fb[(size_t)k * N + i] = 0.0;
            continue;
        }
        for (k = 0; k < q; ++k)
            fa[(size_t)k * N + i] = feq_minus_w(L.w[k], L.c[k], drho[i],
                                                ux[i] + gh[0], uy[i] + gh[1],
                                                uz[i] + gh[2]);
    }
    for (n = 0; n < nsteps; ++n) {
        long z;
#pragma omp parallel for schedule(static)
        for (z = 0; z < nz; ++z) {
            long y, x;
            double fk[QMAX];
            for (y = 0; y < ny; ++y)
                for (x = 0; x < nx; ++x) {
                    long j = x + nx * (y + ny * z);
                    double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, r, vx, vy, vz;
                    int k;
                    if (solid[j]) continue;
                    /* stream (pull) with halfway bounce-back */
                    for (k = 0; k < q; ++k) {
                        long sx = wrap(x - L.c[k][0], nx);
                        long sy = wrap(y - L.c[k][1], ny);
                        long sz = wrap(z - L.c[k][2], nz);
                        long s = sx + nx * (sy + ny * sz);
                        fk[k] = solid[s] ? fa[(size_t)L.opp[k] * N + j]
                                         : fa[(size_t)k * N + s];
                    }
                    /* moments */
                    for (k = 0; k < q; ++k) {
                        d += fk[k];
                        jx += (double)L.c[k][0] * fk[k];
                        jy += (double)L.c[k][1] * fk[k];
                        jz += (double)L.c[k][2] * fk[k];
                    }
                    r = 1.0 / (1.0 + d);
                    drho[j] = d;
                    ux[j] = jx * r + gh[0];
                    uy[j] = jy * r + gh[1];
                    uz[j] = jz * r + gh[2];
                    vx = ux[j] + gh[0];
                    vy = uy[j] + gh[1];
                    vz = uz[j] + gh[2];
                    /* collide */
                    for (k = 0; k < q; ++k)
                        fb[(size_t)k * N + j] =
                            (1.0 - omega) * fk[k]
                            + omega * feq_minus_w(L.w[k], L.c[k], d, vx, vy, vz);
                }
        }
        {
            double *t = fa;
            fa = fb;
            fb = t;
        }
    }
    free(fa);
    free(fb);
    return 0;
}

/* Mass M = sum over fluid nodes of rho = N_fluid + sum drho, and the Darcy
 * permeability k = nu <u_axis> / g_axis with nu = 1/6 and <.> the mean over
 * all N nodes (solid nodes count as zero velocity).  Plain sequential sums in
 * index order. */
int tau1o_reduce(long nx, long ny, long nz, const uint8_t *solid,
                 const double *drho, const double *ux, const double *uy,
                 const double *uz, int axis, double g_axis, double *mass,
                 double *perm)
{
    long N, i, nf = 0;
    double sd = 0.0, su = 0.0;
    const double *ua;
    if (check_args(nx, ny, nz, solid) || axis < 0 || axis > 2) return -1;
    N = nx * ny * nz;
    ua = axis == 0 ? ux : (axis == 1 ? uy : uz);
    for (i = 0; i < N; ++i) {
        if (solid[i]) continue;
        ++nf;
        sd += drho[i];
        su += ua[i];
    }
    if (mass) *mass = (double)nf + sd;
    if (perm) {
        if (g_axis == 0.0) return -1;
        *perm = (1.0 / 6.0) * (su / (double)N) / g_axis;
    }
    return 0;
}
