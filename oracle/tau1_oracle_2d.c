/*
 * tau1_oracle_2d.c -- plain, slow, FP64 CPU oracle for the two-dimensional
 * Tau1 update on D2Q9 with the boundary conditions of the paper's validation
 * runs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite does.  It
 * shares no source, header, table or helper with the GPU path.
 *
 * What it computes (Bacza, Tomczak, Matyka, "The lattice Boltzmann method for
 * fluid flows at relaxation time equal one: performance study"):
 *
 *   * The Tau1 update of Eqs. (8)-(10) on the D2Q9 lattice of the paper's 2-D
 *     kernels: each fluid node receives along c_k the equilibrium of Eq. (3)
 *     of its source node x - c_k, and its new density and momentum are the
 *     sums of those (one reciprocal of the density per node).
 *   * Node types: 0 fluid; 1 wall, halfway bounce-back (Eq. (11)); 2 moving
 *     wall, halfway bounce-back with the wall's momentum added to the
 *     reflected population (the moving lid of the cavity validation):
 *     f_k(x) = f_opp(k)(x) + 6 w_k rho(x) (c_k . u_wall), rho(x) the node's
 *     own previous density.
 *   * Pressure boundaries (the Poiseuille validation, constant-pressure inlet
 *     and outlet): with xbc = 1 the fluid nodes of column x = 0 take the
 *     inlet density rho_in and those of x = nx - 1 the outlet density rho_out.
 *     The populations that would come from outside the box are the unknowns
 *     of the Zou-He reconstruction; the known ones fix the velocity
 *       inlet:  rho_in  u_x = rho_in  - [f0 + f3 + f4 + 2 (f2 + f6 + f8)]
 *       outlet: rho_out u_x = [f0 + f3 + f4 + 2 (f1 + f5 + f7)] - rho_out
 *     (direction numbers below), and the reconstructed node has density
 *     rho_b and velocity (u_x, 0).  At tau = 1 that is the node's new state,
 *     so the Tau1 form needs no population of the boundary node beyond the
 *     known ones.  With f' = f - w_k, whose weights add up to exactly 1 in
 *     both brackets, u_x = (drho_in - S') / rho_in and
 *     u_x = (S' - drho_out) / rho_out.
 *   * Periodic wrap in y, and in x when xbc = 0.  Body force as in the 3-D
 *     oracle: equilibria at v = u + g/2, stored u = j/rho + g/2.
 *
 * Directions: 0 rest; 1 (+1,0), 2 (-1,0), 3 (0,+1), 4 (0,-1), 5 (+1,+1),
 * 6 (-1,-1), 7 (+1,-1), 8 (-1,+1); opp(k) = k+1 for odd k, k-1 for even k > 0.
 * Weights 4/9, 1/9, 1/36 (textbook D2Q9, c_s^2 = 1/3).
 *
 * tau1o2_bgk_run is the brute-force counterpart with full populations (pull
 * streaming, the same wall rules, Zou-He reconstruction of the unknown
 * populations of the pressure nodes, collision (1 - omega) f + omega f_eq).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (never fast-math).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const int C9[9][2] = {{0, 0},  {1, 0},  {-1, 0}, {0, 1},  {0, -1},
                             {1, 1},  {-1, -1}, {1, -1}, {-1, 1}};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static int opp9(int k) { return k == 0 ? 0 : (k % 2 ? k + 1 : k - 1); }

int tau1o2_lattice(int *c, double *w, int *opp)
{
    int k;
    for (k = 0; k < 9; ++k) {
        c[2 * k] = C9[k][0];
        c[2 * k + 1] = C9[k][1];
        w[k] = W9[k];
        opp[k] = opp9(k);
    }
    return 9;
}

static long wrap(long a, long n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* Eq. (3) with c_s^2 = 1/3 minus its weight, direction k, density 1 + ds,
 * velocity v. */
static double feqm(int k, double ds, double vx, double vy)
{
    double rho = 1.0 + ds;
    double cu = (double)C9[k][0] * vx + (double)C9[k][1] * vy;
    double vv = vx * vx + vy * vy;
    double p = (3.0 * cu + (4.5 * cu) * cu) - 1.5 * vv;
    return W9[k] * (ds + rho * p);
}

typedef struct {
    long nx, ny;
    const uint8_t *type;
    double gh[2], uw[2];
    int xbc;
    double din, dout;  /* rho_in - 1, rho_out - 1 */
} grid2_t;

/* Source of direction k at node (x, y): its index, or -1 outside the box
 * (pressure columns only). */
static long source(const grid2_t *G, long x, long y, int k)
{
    long sx = x - C9[k][0];
    long sy = wrap(y - C9[k][1], G->ny);
    if (G->xbc) {
        if (sx < 0 || sx >= G->nx) return -1;
    } else {
        sx = wrap(sx, G->nx);
    }
    return sx + G->nx * sy;
}

/* Arriving value f'_k at fluid node i = (x, y) from source s (a node index):
 * the source's equilibrium, or the bounce-back of the node's own one. */
static double arriving(const grid2_t *G, long i, long s, int k, const double *dr,
                       const double *ux, const double *uy)
{
    if (G->type[s] == 0)
        return feqm(k, dr[s], ux[s] + G->gh[0], uy[s] + G->gh[1]);
    {
        double f = feqm(opp9(k), dr[i], ux[i] + G->gh[0], uy[i] + G->gh[1]);
        if (G->type[s] == 2) {
            double cu = (double)C9[k][0] * G->uw[0] + (double)C9[k][1] * G->uw[1];
            f += 6.0 * W9[k] * (1.0 + dr[i]) * cu;
        }
        return f;
    }
}

/* One Tau1 update of fluid node (x, y); out = drho', ux', uy'. */
static void node2(const grid2_t *G, long x, long y, const double *dr, const double *ux,
                  const double *uy, double out[3])
{
    const long i = x + G->nx * y;
    int k;
    if (G->xbc && (x == 0 || x == G->nx - 1)) {
        /* pressure node: Zou-He velocity from the known populations */
        const int inlet = x == 0;
        const double db = inlet ? G->din : G->dout;
        double f[9] = {0};
        double s;
        for (k = 0; k < 9; ++k) {
            long src = source(G, x, y, k);
            if (src >= 0) f[k] = arriving(G, i, src, k, dr, ux, uy);
        }
        if (inlet) {
            s = (f[0] + f[3] + f[4]) + 2.0 * ((f[2] + f[6]) + f[8]);
            out[1] = (db - s) / (1.0 + db) + G->gh[0];
        } else {
            s = (f[0] + f[3] + f[4]) + 2.0 * ((f[1] + f[5]) + f[7]);
            out[1] = (s - db) / (1.0 + db) + G->gh[0];
        }
        out[0] = db;
        out[2] = G->gh[1];
        return;
    }
    {
        double d = 0.0, jx = 0.0, jy = 0.0, r;
        for (k = 0; k < 9; ++k) {
            const double f = arriving(G, i, source(G, x, y, k), k, dr, ux, uy);
            d += f;
            jx += (double)C9[k][0] * f;
            jy += (double)C9[k][1] * f;
        }
        r = 1.0 / (1.0 + d);
        out[0] = d;
        out[1] = jx * r + G->gh[0];
        out[2] = jy * r + G->gh[1];
    }
}

static int check2(long nx, long ny, const uint8_t *type, int xbc)
{
    long i;
    if (nx < 1 || ny < 1 || !type) return -1;
    if (xbc && nx < 3) return -1;
    for (i = 0; i < nx * ny; ++i)
        if (type[i] > 2) return -1;
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

/* nsteps Tau1 updates in place (state of all nodes; walls are left as they
 * are and never read as sources). */
int tau1o2_run(long nx, long ny, const uint8_t *type, double *drho, double *ux, double *uy,
               const double *g, const double *uw, int xbc, double rho_in, double rho_out,
               long nsteps, int nthreads)
{
    grid2_t G;
    const long n = nx * ny;
    double *nd, *nu, *nv;
    long t;
    if (check2(nx, ny, type, xbc) || nsteps < 0) return -1;
    G.nx = nx;
    G.ny = ny;
    G.type = type;
    G.gh[0] = 0.5 * g[0];
    G.gh[1] = 0.5 * g[1];
    G.uw[0] = uw[0];
    G.uw[1] = uw[1];
    G.xbc = xbc;
    G.din = rho_in - 1.0;
    G.dout = rho_out - 1.0;
    nd = malloc(sizeof(double) * (size_t)n);
    nu = malloc(sizeof(double) * (size_t)n);
    nv = malloc(sizeof(double) * (size_t)n);
    if (!nd || !nu || !nv) {
        free(nd);
        free(nu);
        free(nv);
        return -2;
    }
    set_threads(nthreads);
    for (t = 0; t < nsteps; ++t) {
        long y;
#pragma omp parallel for schedule(static)
        for (y = 0; y < ny; ++y) {
            long x;
            for (x = 0; x < nx; ++x) {
                const long i = x + nx * y;
                double o[3];
                if (type[i]) {
                    nd[i] = drho[i];
                    nu[i] = ux[i];
                    nv[i] = uy[i];
                    continue;
                }
                node2(&G, x, y, drho, ux, uy, o);
                nd[i] = o[0];
                nu[i] = o[1];
                nv[i] = o[2];
            }
        }
        memcpy(drho, nd, sizeof(double) * (size_t)n);
        memcpy(ux, nu, sizeof(double) * (size_t)n);
        memcpy(uy, nv, sizeof(double) * (size_t)n);
    }
    free(nd);
    free(nu);
    free(nv);
    return 0;
}

/* Brute-force LBGK with full populations (stored minus their weights), the
 * same boundary rules, collision (1 - omega) f + omega f_eq; returns the
 * moments after nsteps in drho, ux, uy. */
int tau1o2_bgk_run(long nx, long ny, const uint8_t *type, double *drho, double *ux,
                   double *uy, const double *g, const double *uw, int xbc, double rho_in,
                   double rho_out, double omega, long nsteps)
{
    const long n = nx * ny;
    double *post, *f, *dr;
    double gh[2];
    long t, i;
    int k;
    if (check2(nx, ny, type, xbc) || nsteps < 0) return -1;
    gh[0] = 0.5 * g[0];
    gh[1] = 0.5 * g[1];
    post = malloc(sizeof(double) * 9 * (size_t)n);
    f = malloc(sizeof(double) * 9 * (size_t)n);
    dr = malloc(sizeof(double) * (size_t)n);
    if (!post || !f || !dr) {
        free(post);
        free(f);
        free(dr);
        return -2;
    }
    /* populations after the last collision: equilibria of the initial state */
    for (i = 0; i < n; ++i) {
        dr[i] = drho[i];
        for (k = 0; k < 9; ++k)
            post[9 * i + k] = type[i] ? 0.0 : feqm(k, drho[i], ux[i] + gh[0], uy[i] + gh[1]);
    }
    for (t = 0; t < nsteps; ++t) {
        long y;
        for (y = 0; y < ny; ++y) {
            long x;
            for (x = 0; x < nx; ++x) {
                double *fi = f + 9 * (x + nx * y);
                i = x + nx * y;
                if (type[i]) continue;
                /* pull streaming with the wall rules */
                for (k = 0; k < 9; ++k) {
                    long sx = x - C9[k][0], sy = wrap(y - C9[k][1], ny), s;
                    if (xbc && (sx < 0 || sx >= nx)) {
                        fi[k] = 0.0;  /* unknown: reconstructed below */
                        continue;
                    }
                    s = wrap(sx, nx) + nx * sy;
                    if (type[s] == 0) {
                        fi[k] = post[9 * s + k];
                    } else {
                        fi[k] = post[9 * i + opp9(k)];
                        if (type[s] == 2) {
                            double cu = (double)C9[k][0] * uw[0] + (double)C9[k][1] * uw[1];
                            fi[k] += 6.0 * W9[k] * (1.0 + dr[i]) * cu;
                        }
                    }
                }
                /* Zou-He: the unknown populations of a pressure node */
                if (xbc && (x == 0 || x == nx - 1)) {
                    const int inlet = x == 0;
                    const double db = inlet ? rho_in - 1.0 : rho_out - 1.0;
                    double s, ru;
                    if (inlet) {
                        s = (fi[0] + fi[3] + fi[4]) + 2.0 * ((fi[2] + fi[6]) + fi[8]);
                        ru = db - s;
                        fi[1] = fi[2] + (2.0 / 3.0) * ru;
                        fi[5] = fi[6] - 0.5 * (fi[3] - fi[4]) + ru / 6.0;
                        fi[7] = fi[8] + 0.5 * (fi[3] - fi[4]) + ru / 6.0;
                    } else {
                        s = (fi[0] + fi[3] + fi[4]) + 2.0 * ((fi[1] + fi[5]) + fi[7]);
                        ru = s - db;
                        fi[2] = fi[1] - (2.0 / 3.0) * ru;
                        fi[6] = fi[5] + 0.5 * (fi[3] - fi[4]) - ru / 6.0;
                        fi[8] = fi[7] - 0.5 * (fi[3] - fi[4]) - ru / 6.0;
                    }
                }
            }
        }
        /* moments and collision */
        for (i = 0; i < n; ++i) {
            double d = 0.0, jx = 0.0, jy = 0.0, r, vx, vy;
            double *fi = f + 9 * i;
            if (type[i]) continue;
            for (k = 0; k < 9; ++k) {
                d += fi[k];
                jx += (double)C9[k][0] * fi[k];
                jy += (double)C9[k][1] * fi[k];
            }
            r = 1.0 / (1.0 + d);
            drho[i] = d;
            ux[i] = jx * r + gh[0];
            uy[i] = jy * r + gh[1];
            dr[i] = d;
            vx = ux[i] + gh[0];
            vy = uy[i] + gh[1];
            for (k = 0; k < 9; ++k)
                post[9 * i + k] = (1.0 - omega) * fi[k] + omega * feqm(k, d, vx, vy);
        }
    }
    free(post);
    free(f);
    free(dr);
    return 0;
}

/* Mass sum over fluid nodes of rho, and the mean of u_x over all nodes. */
int tau1o2_reduce(long nx, long ny, const uint8_t *type, const double *drho, const double *ux,
                  double *mass, double *mean_ux)
{
    long i;
    double m = 0.0, s = 0.0;
    if (nx < 1 || ny < 1 || !type) return -1;
    for (i = 0; i < nx * ny; ++i) {
        if (type[i]) continue;
        m += 1.0 + drho[i];
        s += ux[i];
    }
    *mass = m;
    *mean_ux = s / (double)(nx * ny);
    return 0;
}
