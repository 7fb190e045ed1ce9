/*
 * oracle.c -- plain, slow FP64 CPU oracle for the block-adaptive explicit ideal-MHD update.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the CPU-baseline leg of
 * the benchmark load this library. It shares no code, header, table or constant generator with the
 * HIP path, and it is built with contraction and fast-math off (-ffp-contract=off, no -ffast-math).
 *
 * What it computes, following the paper:
 *   - storage: one padded array per block with two ghost layers on every side, variable index
 *     fastest, in the spirit of State_VGB (Sec. 2; Sec. 4.1 sets the ghost width to 2);
 *   - per block (Algorithm 1): face values, face fluxes, source, update; afterwards all ghost cells
 *     are refilled ("exchange messages", Sec. 4.2: copy at equal resolution, restriction from a
 *     finer sender, prolongation from a coarser sender, boundary conditions);
 *   - the equations are ideal MHD in near-conservative form with the eight-wave Powell source
 *     terms, total energy as in Eq. (5), mu0 = 1 (Eqs. 1-5);
 *   - a two-stage time update with a CFL-limited global time step (Sec. 5.1 uses CFL 0.8; Sec. 5.2
 *     contrasts one- and two-stage schemes).
 * Beside the paper's method it holds the learned flux correction of this library (not in the paper):
 * per-face stencil features and a stage that adds given per-face corrections to the plain fluxes, flags
 * cells whose provisional state is not positive or leaves the widened range of its old neighbourhood,
 * and falls back to the plain flux on every face of a flagged cell (or_face_features,
 * or_advance_learned); its network lives in mlp.c.
 * The paper leaves the limiter, reconstruction variables, flux formulas, wave-speed estimate, time-step
 * formula, restriction/prolongation formulas and boundary details unstated; the readings implemented
 * here are listed next to each function.
 *
 * External array layout (inputs and outputs): variable-major U[8][nB][8][8][8], i fastest, float64.
 * Conserved order: rho, rho*ux, rho*uy, rho*uz, Bx, By, Bz, e.
 * Primitive order: rho, ux, uy, uz, Bx, By, Bz, p.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define NC 8              /* cells per block and axis */
#define NGH 2             /* ghost layers */
#define NP (NC + 2 * NGH) /* padded extent: 12 */
#define NV 8
#define NPAD (NP * NP * NP)

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_INFLOW = 2 };
enum { REL_SAME = 0, REL_COARSER = 1, REL_FINER = 2, REL_OUTFLOW = -1, REL_INFLOW = -2 };
enum { FLUX_RUSANOV = 0, FLUX_HLLE = 1, FLUX_LINDE = 2 };

static const double GAM = 5.0 / 3.0;

typedef struct {
    int32_t nroot[3];
    double origin[3];
    double dx0;
    int32_t bc[6];
    double inflow_w[8];
    double body_c[3];
    double body_r;
} or_sim;

typedef struct {
    int32_t flux;      /* FLUX_RUSANOV, FLUX_HLLE or FLUX_LINDE */
    int32_t powell;    /* 0 / 1 */
    int32_t n_table;   /* number of stages in the table (1 or 2) */
    int32_t recompute_dt;
    double alpha[2];
    double beta[2];
    double cfl;
    int32_t local_dt;  /* 1: local time stepping, dt[] holds one dt per cell ([nB][8][8][8]) */
} or_opts;

typedef struct {
    int nb, ns;
    int32_t *level, *ijk, *sim;
    or_sim *sims;
    int32_t **lut; /* lut[2*s + l]: block id at block coordinates of level l, or -1 */
} or_grid;

/* ------------------------------------------------------------------------------------------------ */
/* state conversions (Eq. 5 with mu0 = 1)                                                            */

void or_prim_to_cons(const double *w, double *u)
{
    double rho = w[0];
    double u2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    double b2 = w[4] * w[4] + w[5] * w[5] + w[6] * w[6];
    u[0] = rho;
    u[1] = rho * w[1];
    u[2] = rho * w[2];
    u[3] = rho * w[3];
    u[4] = w[4];
    u[5] = w[5];
    u[6] = w[6];
    u[7] = w[7] / (GAM - 1.0) + 0.5 * rho * u2 + 0.5 * b2;
}

void or_cons_to_prim(const double *u, double *w)
{
    double rho = u[0];
    double ux = u[1] / rho, uy = u[2] / rho, uz = u[3] / rho;
    double u2 = ux * ux + uy * uy + uz * uz;
    double b2 = u[4] * u[4] + u[5] * u[5] + u[6] * u[6];
    w[0] = rho;
    w[1] = ux;
    w[2] = uy;
    w[3] = uz;
    w[4] = u[4];
    w[5] = u[5];
    w[6] = u[6];
    w[7] = (GAM - 1.0) * (u[7] - 0.5 * rho * u2 - 0.5 * b2);
}

/* Physical flux along axis d of the conservation laws Eqs. (1)-(4) (left-hand sides). */
void or_phys_flux(const double *w, int d, double *f)
{
    double rho = w[0], p = w[7];
    const double *uv = w + 1, *bv = w + 4;
    double un = uv[d], bn = bv[d];
    double u2 = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
    double b2 = bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2];
    double ub = uv[0] * bv[0] + uv[1] * bv[1] + uv[2] * bv[2];
    double ptot = p + 0.5 * b2;
    double e = p / (GAM - 1.0) + 0.5 * rho * u2 + 0.5 * b2;
    f[0] = rho * un;
    for (int a = 0; a < 3; a++) {
        f[1 + a] = rho * uv[a] * un - bv[a] * bn;
        if (a == d) f[1 + a] += ptot;
        f[4 + a] = un * bv[a] - bn * uv[a];
    }
    f[7] = un * (e + ptot) - bn * ub;
}

/* Fast magnetosonic speed along axis d: the largest root of the ideal-MHD dispersion relation,
 * c_f^2 = ((a^2 + b^2) + sqrt((a^2 + b^2)^2 - 4 a^2 b_n^2)) / 2 with a^2 = gamma p / rho,
 * b^2 = |B|^2 / rho, b_n^2 = B_d^2 / rho. For k perpendicular to B it reduces to the paper's
 * c_F = sqrt(c_s^2 + v_A^2) (Sec. 5.1). */
double or_fast_speed(const double *w, int d)
{
    double rho = w[0];
    double a2 = GAM * w[7] / rho;
    double b2 = (w[4] * w[4] + w[5] * w[5] + w[6] * w[6]) / rho;
    double bn2 = w[4 + d] * w[4 + d] / rho;
    double s = a2 + b2;
    double disc = s * s - 4.0 * a2 * bn2;
    if (disc < 0.0) disc = 0.0;
    return sqrt(0.5 * (s + sqrt(disc)));
}

/* Numerical flux from primitive face states (reading: Rusanov with the larger of the two |u_n|+c_f;
 * HLLE with Davis-type min/max signal speeds; every component, B_n included, gets the same
 * dissipation).
 *
 * FLUX_LINDE, the flux the paper's fast-wave test names (Sec. 5.1) without printing it; reading, after
 * T. Linde's two-state HLL solver (Int. J. Numer. Meth. Fluids 40, 2002), whose aim is that HLL's
 * dissipation vanish on an isolated intermediate discontinuity: HLLE plus an anti-diffusion term for the
 * entropy (contact) wave. Its density jump is delta = minmod(drho - dp / c^2, drho) with
 * c^2 = gamma (p_L + p_R) / (rho_L + rho_R) (the part of the density jump no pressure change explains,
 * never larger than the jump itself), its conserved jump dU_c = delta (1, u_bar, 0, 0, 0, |u_bar|^2 / 2)
 * at the mean velocity u_bar, and the term replaces HLL's dissipation of that jump by upwinding at the
 * contact speed lambda = u_bar_n clamped to [S_L, S_R]:
 *   F = F_HLLE + K dU_c / (S_R - S_L),   K = -S_L S_R + S_L max(lambda, 0) + S_R min(lambda, 0) >= 0.
 * An isolated contact (u, p, B continuous, rho jumping) gets the exact upwind flux, F_L for lambda >= 0
 * and F_R otherwise; where S_L >= 0 or S_R <= 0 the flux is HLLE's (upwind). */
void or_num_flux(const double *wl, const double *wr, int d, int kind, double *f)
{
    double ul[8], ur[8], fl[8], fr[8];
    or_prim_to_cons(wl, ul);
    or_prim_to_cons(wr, ur);
    or_phys_flux(wl, d, fl);
    or_phys_flux(wr, d, fr);
    double cl = or_fast_speed(wl, d), cr = or_fast_speed(wr, d);
    double unl = wl[1 + d], unr = wr[1 + d];
    if (kind == FLUX_RUSANOV) {
        double cmax = fmax(fabs(unl) + cl, fabs(unr) + cr);
        for (int v = 0; v < 8; v++) f[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * cmax * (ur[v] - ul[v]);
    } else {
        double sl = fmin(unl - cl, unr - cr);
        double sr = fmax(unl + cl, unr + cr);
        if (sl >= 0.0) {
            for (int v = 0; v < 8; v++) f[v] = fl[v];
        } else if (sr <= 0.0) {
            for (int v = 0; v < 8; v++) f[v] = fr[v];
        } else {
            double duc[8] = {0, 0, 0, 0, 0, 0, 0, 0}, K = 0.0;
            if (kind == FLUX_LINDE) {
                double drho = wr[0] - wl[0], dp = wr[7] - wl[7];
                double c2 = GAM * (wl[7] + wr[7]) / (wl[0] + wr[0]);
                double t = drho - dp / c2, delta = 0.0;
                if (t > 0.0 && drho > 0.0) delta = fmin(t, drho);
                if (t < 0.0 && drho < 0.0) delta = fmax(t, drho);
                double ub[3], ub2 = 0.0;
                for (int a = 0; a < 3; a++) {
                    ub[a] = 0.5 * (wl[1 + a] + wr[1 + a]);
                    ub2 += ub[a] * ub[a];
                }
                double lam = fmin(fmax(ub[d], sl), sr);
                K = -sl * sr + sl * fmax(lam, 0.0) + sr * fmin(lam, 0.0);
                duc[0] = delta;
                for (int a = 0; a < 3; a++) duc[1 + a] = delta * ub[a];
                duc[7] = delta * 0.5 * ub2;
            }
            for (int v = 0; v < 8; v++)
                f[v] = (sr * fl[v] - sl * fr[v] + sl * sr * (ur[v] - ul[v]) + K * duc[v]) / (sr - sl);
        }
    }
}

/* ------------------------------------------------------------------------------------------------ */
/* limiters                                                                                         */

static double minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}

static double minmod2(double a, double b)
{
    if (a > 0.0 && b > 0.0) return fmin(a, b);
    if (a < 0.0 && b < 0.0) return fmax(a, b);
    return 0.0;
}

/* Monotonized-central limited slope of the middle value (the paper's "second-order scheme" leaves the
 * limiter open; MC is the reading): minmod(2 D-, (D- + D+)/2, 2 D+). */
double or_mc_slope(double wm, double w0, double wp)
{
    double dm = w0 - wm, dp = wp - w0;
    return minmod3(2.0 * dm, 0.5 * (dm + dp), 2.0 * dp);
}

/* Restriction: pairwise-tree mean of the 8 fine children c[z][y][x] (x fastest). */
double or_restrict8(const double *c)
{
    return (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]))) * 0.125;
}

/* Prolongation of one variable: coarse value plus a quarter of the minmod slope per axis, with the sign
 * of the fine cell's half, added in the order x, y, z. cm/cp are the coarse neighbours. */
double or_prolong1(double uc, const double *cm, const double *cp, const int *s)
{
    double v = uc;
    for (int d = 0; d < 3; d++) {
        double sig = minmod2(uc - cm[d], cp[d] - uc);
        v = v + 0.25 * (double)s[d] * sig;
    }
    return v;
}

/* ------------------------------------------------------------------------------------------------ */
/* grid                                                                                             */

static long nblk_axis(const or_sim *s, int l, int a) { return (long)s->nroot[a] << l; }
static long ncell_axis(const or_sim *s, int l, int a) { return nblk_axis(s, l, a) * NC; }

static int lut_get(const or_grid *g, int s, int l, const long bb[3])
{
    const or_sim *sm = &g->sims[s];
    long nx = nblk_axis(sm, l, 0), ny = nblk_axis(sm, l, 1), nz = nblk_axis(sm, l, 2);
    if (bb[0] < 0 || bb[1] < 0 || bb[2] < 0 || bb[0] >= nx || bb[1] >= ny || bb[2] >= nz) return -1;
    return g->lut[2 * s + l][(bb[2] * ny + bb[1]) * nx + bb[0]];
}

void or_grid_free(or_grid *g)
{
    if (!g) return;
    if (g->lut)
        for (int i = 0; i < 2 * g->ns; i++) free(g->lut[i]);
    free(g->lut);
    free(g->level);
    free(g->ijk);
    free(g->sim);
    free(g->sims);
    free(g);
}

/* Returns NULL on an invalid grid: levels outside {0,1}, blocks outside the root box, overlaps, or a
 * root region that is neither one level-0 block nor fully covered by its 8 level-1 children. */
or_grid *or_grid_create(int nb, const int32_t *level, const int32_t *ijk, const int32_t *sim, int ns,
                        const or_sim *sims)
{
    or_grid *g = calloc(1, sizeof(or_grid));
    g->nb = nb;
    g->ns = ns;
    g->level = malloc(sizeof(int32_t) * (size_t)nb);
    g->ijk = malloc(sizeof(int32_t) * 3 * (size_t)nb);
    g->sim = malloc(sizeof(int32_t) * (size_t)nb);
    g->sims = malloc(sizeof(or_sim) * (size_t)ns);
    memcpy(g->level, level, sizeof(int32_t) * (size_t)nb);
    memcpy(g->ijk, ijk, sizeof(int32_t) * 3 * (size_t)nb);
    memcpy(g->sim, sim, sizeof(int32_t) * (size_t)nb);
    memcpy(g->sims, sims, sizeof(or_sim) * (size_t)ns);
    g->lut = calloc(2 * (size_t)ns, sizeof(int32_t *));
    for (int s = 0; s < ns; s++)
        for (int l = 0; l < 2; l++) {
            long n = nblk_axis(&sims[s], l, 0) * nblk_axis(&sims[s], l, 1) * nblk_axis(&sims[s], l, 2);
            g->lut[2 * s + l] = malloc(sizeof(int32_t) * (size_t)n);
            for (long i = 0; i < n; i++) g->lut[2 * s + l][i] = -1;
        }
    for (int b = 0; b < nb; b++) {
        int s = sim[b], l = level[b];
        if (s < 0 || s >= ns || l < 0 || l > 1) goto bad;
        const or_sim *sm = &sims[s];
        long nx = nblk_axis(sm, l, 0), ny = nblk_axis(sm, l, 1), nz = nblk_axis(sm, l, 2);
        long i = ijk[3 * b], j = ijk[3 * b + 1], k = ijk[3 * b + 2];
        if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) goto bad;
        int32_t *slot = &g->lut[2 * s + l][(k * ny + j) * nx + i];
        if (*slot != -1) goto bad;
        *slot = b;
    }
    /* coverage: each root is a leaf or has all 8 children */
    for (int s = 0; s < ns; s++) {
        const or_sim *sm = &sims[s];
        for (long k = 0; k < sm->nroot[2]; k++)
            for (long j = 0; j < sm->nroot[1]; j++)
                for (long i = 0; i < sm->nroot[0]; i++) {
                    long r[3] = {i, j, k};
                    int leaf = lut_get(g, s, 0, r) >= 0;
                    int nch = 0;
                    for (int c = 0; c < 8; c++) {
                        long cc[3] = {2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1)};
                        nch += lut_get(g, s, 1, cc) >= 0;
                    }
                    if (!((leaf && nch == 0) || (!leaf && nch == 8))) goto bad;
                }
    }
    return g;
bad:
    or_grid_free(g);
    return NULL;
}

/* Neighbour table: for block b and direction index n (dx, dy, dz in {-1,0,1}^3 minus 0, enumerated
 * with dx fastest, the zero vector skipped), five ints {relation, id0..id3}. Relation: 0 same level,
 * 1 coarser, 2 finer (the finer blocks touching b, enumerated x fastest over the free sub-positions),
 * -1 outflow / -2 inflow when the direction leaves the domain through a non-periodic face (the first
 * such axis in the order x, y, z decides). Unused ids are -1. */
void or_neighbors(const or_grid *g, int32_t *out)
{
    for (int b = 0; b < g->nb; b++) {
        int s = g->sim[b], l = g->level[b];
        const or_sim *sm = &g->sims[s];
        int n = 0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    int32_t *e = out + ((size_t)b * 26 + n) * 5;
                    n++;
                    for (int q = 0; q < 5; q++) e[q] = -1;
                    int dd[3] = {dx, dy, dz};
                    long nbk[3];
                    int boundary = 0;
                    for (int a = 0; a < 3 && !boundary; a++) {
                        long N = nblk_axis(sm, l, a);
                        long c = g->ijk[3 * b + a] + dd[a];
                        if (c < 0 || c >= N) {
                            int t = sm->bc[2 * a + (c < 0 ? 0 : 1)];
                            if (t == BC_PERIODIC) c = (c + N) % N;
                            else {
                                e[0] = t == BC_OUTFLOW ? REL_OUTFLOW : REL_INFLOW;
                                boundary = 1;
                            }
                        }
                        nbk[a] = c;
                    }
                    if (boundary) continue;
                    int id = lut_get(g, s, l, nbk);
                    if (id >= 0) {
                        e[0] = REL_SAME;
                        e[1] = id;
                        continue;
                    }
                    if (l == 1) {
                        long cb[3] = {nbk[0] / 2, nbk[1] / 2, nbk[2] / 2};
                        id = lut_get(g, s, 0, cb);
                        if (id >= 0) {
                            e[0] = REL_COARSER;
                            e[1] = id;
                        }
                        continue;
                    }
                    e[0] = REL_FINER;
                    int m = 1;
                    for (int sz = 0; sz < 2; sz++)
                        for (int sy = 0; sy < 2; sy++)
                            for (int sx = 0; sx < 2; sx++) {
                                int sub[3] = {sx, sy, sz};
                                int ok = 1;
                                for (int a = 0; a < 3; a++) {
                                    if (dd[a] == 1 && sub[a] != 0) ok = 0;
                                    if (dd[a] == -1 && sub[a] != 1) ok = 0;
                                }
                                if (!ok) continue;
                                long fb[3] = {2 * nbk[0] + sx, 2 * nbk[1] + sy, 2 * nbk[2] + sz};
                                e[m++] = lut_get(g, s, 1, fb);
                            }
                }
    }
}

/* ------------------------------------------------------------------------------------------------ */
/* padded block storage: st[b][k][j][i][v], i, j, k in [0, 12), interior at [2, 10)                  */

#define PIDX(i, j, k) ((((size_t)(k)) * NP + (size_t)(j)) * NP + (size_t)(i))

static double *pad_alloc(int nb) { return calloc((size_t)nb * NPAD * NV, sizeof(double)); }

static double *pcell(double *st, int b, int i, int j, int k) /* i,j,k in block coordinates [-2,10) */
{
    return st + ((size_t)b * NPAD + PIDX(i + NGH, j + NGH, k + NGH)) * NV;
}

static void pad_from_ext(const or_grid *g, const double *U, double *st)
{
    size_t nbc = (size_t)g->nb * 512;
    for (int b = 0; b < g->nb; b++)
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    double *c = pcell(st, b, i, j, k);
                    for (int v = 0; v < NV; v++) c[v] = U[v * nbc + (size_t)b * 512 + (k * 8 + j) * 8 + i];
                }
}

static void pad_to_ext(const or_grid *g, double *st, double *U)
{
    size_t nbc = (size_t)g->nb * 512;
    for (int b = 0; b < g->nb; b++)
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    double *c = pcell(st, b, i, j, k);
                    for (int v = 0; v < NV; v++) U[v * nbc + (size_t)b * 512 + (k * 8 + j) * 8 + i] = c[v];
                }
}

/* ------------------------------------------------------------------------------------------------ */
/* ghost values (exchange of messages between blocks, Sec. 4.2)                                     */

/* Boundary handling of a level-l global cell index, axis by axis in the order x, y, z: periodic wraps,
 * outflow clamps to the nearest interior cell along the normal, inflow returns 1. */
static int apply_bc(const or_grid *g, int s, int l, long G[3])
{
    const or_sim *sm = &g->sims[s];
    for (int a = 0; a < 3; a++) {
        long N = ncell_axis(sm, l, a);
        if (G[a] >= 0 && G[a] < N) continue;
        int side = G[a] < 0 ? 0 : 1;
        int t = sm->bc[2 * a + side];
        if (t == BC_PERIODIC) G[a] = ((G[a] % N) + N) % N;
        else if (t == BC_OUTFLOW) G[a] = side ? N - 1 : 0;
        else return 1;
    }
    return 0;
}

static void inflow_cons(const or_grid *g, int s, double *u) { or_prim_to_cons(g->sims[s].inflow_w, u); }

/* interior value of the leaf that holds level-l cell G (in-domain), for levels where a leaf exists */
static int leaf_value(const or_grid *g, const double *st, int s, int l, const long G[3], double *u)
{
    long bb[3] = {G[0] / NC, G[1] / NC, G[2] / NC};
    int b = lut_get(g, s, l, bb);
    if (b < 0) return 0;
    const double *c = pcell((double *)st, b, (int)(G[0] % NC), (int)(G[1] % NC), (int)(G[2] % NC));
    memcpy(u, c, sizeof(double) * NV);
    return 1;
}

/* Restriction of level-0 cell G from the 8 level-1 cells 2G + {0,1}^3. */
static int restricted_value(const or_grid *g, const double *st, int s, const long G[3], double *u)
{
    double c[8][NV];
    for (int q = 0; q < 8; q++) {
        long F[3] = {2 * G[0] + (q & 1), 2 * G[1] + ((q >> 1) & 1), 2 * G[2] + ((q >> 2) & 1)};
        if (!leaf_value(g, st, s, 1, F, c[q])) return 0;
    }
    for (int v = 0; v < NV; v++) {
        double cv[8];
        for (int q = 0; q < 8; q++) cv[q] = c[q][v];
        u[v] = (((cv[0] + cv[1]) + (cv[2] + cv[3])) + ((cv[4] + cv[5]) + (cv[6] + cv[7]))) * 0.125;
    }
    return 1;
}

/* Level-0 ("pass-1") value at a possibly out-of-domain level-0 index: boundary rule, then a level-0
 * leaf's interior, else restriction from level 1. */
static void coarse_value(const or_grid *g, const double *st, int s, long G[3], double *u)
{
    if (apply_bc(g, s, 0, G)) {
        inflow_cons(g, s, u);
        return;
    }
    if (leaf_value(g, st, s, 0, G, u)) return;
    if (restricted_value(g, st, s, G, u)) return;
    fprintf(stderr, "oracle: uncovered coarse cell\n");
    abort();
}

/* Ghost value of a level-l cell at global index G (may be outside the domain). */
static void ghost_value(const or_grid *g, const double *st, int s, int l, const long G0[3], double *u)
{
    long G[3] = {G0[0], G0[1], G0[2]};
    if (apply_bc(g, s, l, G)) {
        inflow_cons(g, s, u);
        return;
    }
    if (leaf_value(g, st, s, l, G, u)) return;
    if (l == 0) {
        if (restricted_value(g, st, s, G, u)) return;
    } else {
        /* prolongation from the coarse cell C = floor(G / 2) */
        long C[3] = {G[0] / 2, G[1] / 2, G[2] / 2};
        double uc[NV], um[3][NV], up[3][NV];
        if (!leaf_value(g, st, s, 0, C, uc)) {
            fprintf(stderr, "oracle: prolongation source missing\n");
            abort();
        }
        for (int d = 0; d < 3; d++) {
            long Cm[3] = {C[0], C[1], C[2]}, Cp[3] = {C[0], C[1], C[2]};
            Cm[d] -= 1;
            Cp[d] += 1;
            coarse_value(g, st, s, Cm, um[d]);
            coarse_value(g, st, s, Cp, up[d]);
        }
        int sg[3];
        for (int d = 0; d < 3; d++) sg[d] = (G[d] & 1) ? 1 : -1;
        for (int v = 0; v < NV; v++) {
            double cm[3] = {um[0][v], um[1][v], um[2][v]};
            double cp[3] = {up[0][v], up[1][v], up[2][v]};
            u[v] = or_prolong1(uc[v], cm, cp, sg);
        }
        return;
    }
    fprintf(stderr, "oracle: uncovered cell\n");
    abort();
}

/* Fill every ghost cell of every block (faces, edges and corners). */
static void exchange_messages(const or_grid *g, double *st)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < g->nb; b++) {
        int s = g->sim[b], l = g->level[b];
        for (int k = -NGH; k < NC + NGH; k++)
            for (int j = -NGH; j < NC + NGH; j++)
                for (int i = -NGH; i < NC + NGH; i++) {
                    if (i >= 0 && i < NC && j >= 0 && j < NC && k >= 0 && k < NC) continue;
                    long G[3] = {(long)g->ijk[3 * b] * NC + i, (long)g->ijk[3 * b + 1] * NC + j,
                                 (long)g->ijk[3 * b + 2] * NC + k};
                    ghost_value(g, st, s, l, G, pcell(st, b, i, j, k));
                }
    }
}

/* ------------------------------------------------------------------------------------------------ */
/* body mask: a cell belongs to the body when its centre lies strictly inside the sphere             */

static double cell_dx(const or_grid *g, int b) { return g->sims[g->sim[b]].dx0 / (double)(1 << g->level[b]); }

static int is_body(const or_grid *g, int b, int i, int j, int k)
{
    const or_sim *sm = &g->sims[g->sim[b]];
    if (!(sm->body_r > 0.0)) return 0;
    double dx = cell_dx(g, b);
    int ii[3] = {i, j, k};
    double r2 = 0.0;
    for (int a = 0; a < 3; a++) {
        long G = (long)g->ijk[3 * b + a] * NC + ii[a];
        double x = sm->origin[a] + ((double)G + 0.5) * dx;
        double t = x - sm->body_c[a];
        r2 = r2 + t * t;
    }
    return r2 < sm->body_r * sm->body_r;
}

/* ------------------------------------------------------------------------------------------------ */
/* time step                                                                                        */

/* dt = CFL * min over fluid cells of 1 / sum_d ((|u_d| + c_f,d) / dx_d), per simulation. */
static void compute_dt(const or_grid *g, double *st, double cfl, double *dt)
{
    for (int s = 0; s < g->ns; s++) dt[s] = INFINITY;
    for (int b = 0; b < g->nb; b++) {
        int s = g->sim[b];
        double dx = cell_dx(g, b);
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    if (is_body(g, b, i, j, k)) continue;
                    double w[NV];
                    or_cons_to_prim(pcell(st, b, i, j, k), w);
                    double lam = 0.0;
                    for (int d = 0; d < 3; d++) lam = lam + (fabs(w[1 + d]) + or_fast_speed(w, d)) / dx;
                    double t = cfl * (1.0 / lam);
                    if (t < dt[s]) dt[s] = t;
                }
    }
}

/* Local time stepping (the paper's steady-state sessions, Sec. 5.2): every fluid cell advances with its
 * own step, the same CFL bound as compute_dt taken per cell, dt_i = CFL * 1 / sum_d ((|u_d| + c_f,d) / dx).
 * Body cells get 0 (they are not updated). dt[] has the layout of one variable, [nB][8][8][8]. */
static void compute_local_dt(const or_grid *g, double *st, double cfl, double *dt)
{
    for (int b = 0; b < g->nb; b++) {
        double dx = cell_dx(g, b);
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    double *t = dt + (size_t)b * NC * NC * NC + (k * NC + j) * NC + i;
                    if (is_body(g, b, i, j, k)) {
                        *t = 0.0;
                        continue;
                    }
                    double w[NV];
                    or_cons_to_prim(pcell(st, b, i, j, k), w);
                    double lam = 0.0;
                    for (int d = 0; d < 3; d++) lam = lam + (fabs(w[1 + d]) + or_fast_speed(w, d)) / dx;
                    *t = cfl * (1.0 / lam);
                }
    }
}

/* ------------------------------------------------------------------------------------------------ */
/* one stage on one block (Algorithm 1, body of the block loop)                                     */

typedef struct {
    double f[3][NC + 1][NC][NC][NV]; /* face fluxes: [axis][face index along axis][t2][t1][v] */
    double bbar[3][NC + 1][NC][NC];  /* average normal B at the face */
} or_faces;

static void face_cell(int d, int f, int t1, int t2, int *ijk)
{
    /* cell with index f along axis d and transverse indices (t1, t2) along the other axes in order */
    int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
    ijk[d] = f;
    ijk[a1] = t1;
    ijk[a2] = t2;
}

static void calc_face_values_and_fluxes(const or_grid *g, int b, double *st, const or_opts *o, or_faces *F)
{
    for (int d = 0; d < 3; d++)
        for (int t2 = 0; t2 < NC; t2++)
            for (int t1 = 0; t1 < NC; t1++)
                for (int f = 0; f <= NC; f++) {
                    /* face f lies between cells f-1 (left) and f (right) along axis d */
                    int c[4][3];
                    for (int q = 0; q < 4; q++) face_cell(d, f - 2 + q, t1, t2, c[q]);
                    double w[4][NV];
                    int body[4];
                    for (int q = 0; q < 4; q++) {
                        or_cons_to_prim(pcell(st, b, c[q][0], c[q][1], c[q][2]), w[q]);
                        body[q] = is_body(g, b, c[q][0], c[q][1], c[q][2]);
                    }
                    double wl[NV], wr[NV], *fv = F->f[d][f][t2][t1];
                    if (body[1] && body[2]) {
                        for (int v = 0; v < NV; v++) fv[v] = 0.0;
                        F->bbar[d][f][t2][t1] = 0.0;
                        continue;
                    }
                    if (body[2]) { /* reflecting wall on the right: mirror of the first-order left state */
                        memcpy(wl, w[1], sizeof wl);
                        memcpy(wr, wl, sizeof wr);
                        wr[1 + d] = -wl[1 + d];
                    } else if (body[1]) {
                        memcpy(wr, w[2], sizeof wr);
                        memcpy(wl, wr, sizeof wl);
                        wl[1 + d] = -wr[1 + d];
                    } else {
                        for (int v = 0; v < NV; v++) {
                            double sl = (body[0] || body[2]) ? 0.0 : or_mc_slope(w[0][v], w[1][v], w[2][v]);
                            double sr = (body[1] || body[3]) ? 0.0 : or_mc_slope(w[1][v], w[2][v], w[3][v]);
                            wl[v] = w[1][v] + 0.5 * sl;
                            wr[v] = w[2][v] - 0.5 * sr;
                        }
                    }
                    or_num_flux(wl, wr, d, o->flux, fv);
                    F->bbar[d][f][t2][t1] = 0.5 * (wl[4 + d] + wr[4 + d]);
                }
}

/* Source (Powell terms, right-hand sides of Eqs. 2-4) and update of the physical cells.
 * out = alpha * u0 + (1 - alpha) * in + beta * dt * (-sum_d dF_d / dx + S). Body cells are copied.
 * dloc (may be NULL): the block's per-cell dt under local time stepping, in place of dt. */
static void calc_source_and_update(const or_grid *g, int b, double *in, double *u0, double *out, double dt,
                                   const double *dloc, double alpha, double beta, const or_opts *o,
                                   const or_faces *F)
{
    double dx = cell_dx(g, b);
    for (int k = 0; k < NC; k++)
        for (int j = 0; j < NC; j++)
            for (int i = 0; i < NC; i++) {
                double *ci = pcell(in, b, i, j, k), *c0 = pcell(u0, b, i, j, k), *co = pcell(out, b, i, j, k);
                if (is_body(g, b, i, j, k)) {
                    for (int v = 0; v < NV; v++) co[v] = ci[v];
                    continue;
                }
                int ii[3] = {i, j, k};
                double rhs[NV] = {0};
                double divb = 0.0;
                for (int d = 0; d < 3; d++) {
                    int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
                    int f = ii[d], t1 = ii[a1], t2 = ii[a2];
                    for (int v = 0; v < NV; v++)
                        rhs[v] = rhs[v] - (F->f[d][f + 1][t2][t1][v] - F->f[d][f][t2][t1][v]) / dx;
                    divb = divb + (F->bbar[d][f + 1][t2][t1] - F->bbar[d][f][t2][t1]) / dx;
                }
                if (o->powell) {
                    double w[NV];
                    or_cons_to_prim(ci, w);
                    double ub = w[1] * w[4] + w[2] * w[5] + w[3] * w[6];
                    for (int a = 0; a < 3; a++) {
                        rhs[1 + a] = rhs[1 + a] - divb * w[4 + a];
                        rhs[4 + a] = rhs[4 + a] - divb * w[1 + a];
                    }
                    rhs[7] = rhs[7] - divb * ub;
                }
                double dtc = dloc ? dloc[(k * NC + j) * NC + i] : dt;
                for (int v = 0; v < NV; v++)
                    co[v] = alpha * c0[v] + (1.0 - alpha) * ci[v] + beta * dtc * rhs[v];
            }
}

/* ------------------------------------------------------------------------------------------------ */
/* flux correction at resolution changes: the coarse cell next to a coarse-fine face replaces its     */
/* coarse flux by the pairwise mean of the four fine fluxes covering that face                      */

static int find_fine_faces(const or_grid *g, int s, int bc, int d, int side, int fine_ids[4])
{
    /* the four level-1 blocks across face (d, side) of level-0 block bc, ordered by (t1, t2) with t1
     * fastest, where t1 < t2 are the two axes other than d */
    const or_sim *sm = &g->sims[s];
    long nb[3];
    for (int a = 0; a < 3; a++) nb[a] = g->ijk[3 * bc + a];
    nb[d] += side ? 1 : -1;
    long N = nblk_axis(sm, 0, d);
    if (nb[d] < 0 || nb[d] >= N) {
        if (sm->bc[2 * d + side] != BC_PERIODIC) return 0;
        nb[d] = (nb[d] + N) % N;
    }
    if (lut_get(g, s, 0, nb) >= 0) return 0;
    int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
    int q = 0;
    for (int s2 = 0; s2 < 2; s2++)
        for (int s1 = 0; s1 < 2; s1++) {
            long fb[3];
            fb[d] = 2 * nb[d] + (side ? 0 : 1);
            fb[a1] = 2 * nb[a1] + s1;
            fb[a2] = 2 * nb[a2] + s2;
            fine_ids[q++] = lut_get(g, s, 1, fb);
        }
    return 1;
}

/* dt: per simulation, or per cell when local (local time stepping) */
static void flux_correction(const or_grid *g, or_faces **faces, double *out, const double *dt, int local,
                            double beta)
{
    for (int b = 0; b < g->nb; b++) {
        if (g->level[b] != 0 || !faces[b]) continue;
        int s = g->sim[b];
        double dxc = cell_dx(g, b);
        for (int d = 0; d < 3; d++)
            for (int side = 0; side < 2; side++) {
                int fid[4];
                if (!find_fine_faces(g, s, b, d, side, fid)) continue;
                int fc = side ? NC : 0;         /* coarse face index along d */
                int ff = side ? 0 : NC;         /* the same face seen from the fine blocks */
                double sgn = side ? 1.0 : -1.0;
                for (int t2 = 0; t2 < NC; t2++)
                    for (int t1 = 0; t1 < NC; t1++) {
                        /* fine block covering this coarse face cell, and its first fine face index */
                        int q = (t1 / 4) + 2 * (t2 / 4);
                        const or_faces *Ff = faces[fid[q]];
                        int f1 = 2 * (t1 % 4), f2 = 2 * (t2 % 4);
                        int ci[3];
                        face_cell(d, side ? NC - 1 : 0, t1, t2, ci);
                        double *co = pcell(out, b, ci[0], ci[1], ci[2]);
                        if (is_body(g, b, ci[0], ci[1], ci[2])) continue;
                        double dtc = local ? dt[(size_t)b * NC * NC * NC + (ci[2] * NC + ci[1]) * NC + ci[0]] : dt[s];
                        for (int v = 0; v < NV; v++) {
                            double a = Ff->f[d][ff][f2][f1][v], bq = Ff->f[d][ff][f2][f1 + 1][v];
                            double c = Ff->f[d][ff][f2 + 1][f1][v], e = Ff->f[d][ff][f2 + 1][f1 + 1][v];
                            double fmean = ((a + bq) + (c + e)) * 0.25;
                            double fcv = faces[b]->f[d][fc][t2][t1][v];
                            co[v] = co[v] + beta * dtc * sgn * (fcv - fmean) / dxc;
                        }
                    }
            }
    }
}

static int has_level_change(const or_grid *g, int b)
{
    int s = g->sim[b], l = g->level[b];
    const or_sim *sm = &g->sims[s];
    for (int d = 0; d < 3; d++)
        for (int side = 0; side < 2; side++) {
            long nb[3];
            for (int a = 0; a < 3; a++) nb[a] = g->ijk[3 * b + a];
            nb[d] += side ? 1 : -1;
            long N = nblk_axis(sm, l, d);
            if (nb[d] < 0 || nb[d] >= N) {
                if (sm->bc[2 * d + side] != BC_PERIODIC) continue;
                nb[d] = (nb[d] + N) % N;
            }
            if (lut_get(g, s, l, nb) < 0) return 1;
        }
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* public driver                                                                                     */

/* Primitive to conserved over all interior cells (external layout). */
void or_set_state(const or_grid *g, const double *W, double *U)
{
    size_t nc = (size_t)g->nb * 512;
    for (size_t c = 0; c < nc; c++) {
        double w[NV], u[NV];
        for (int v = 0; v < NV; v++) w[v] = W[v * nc + c];
        or_prim_to_cons(w, u);
        for (int v = 0; v < NV; v++) U[v * nc + c] = u[v];
    }
}

/* Every ghost cell of every block into view[8][nB][12][12][12] (interior copied too). */
void or_fill_ghosts(const or_grid *g, const double *U, double *view)
{
    double *st = pad_alloc(g->nb);
    pad_from_ext(g, U, st);
    exchange_messages(g, st);
    size_t nbp = (size_t)g->nb * NPAD;
    for (int b = 0; b < g->nb; b++)
        for (size_t c = 0; c < NPAD; c++)
            for (int v = 0; v < NV; v++) view[v * nbp + (size_t)b * NPAD + c] = st[((size_t)b * NPAD + c) * NV + v];
    free(st);
}

void or_dt(const or_grid *g, const double *U, double cfl, double *dt)
{
    double *st = pad_alloc(g->nb);
    pad_from_ext(g, U, st);
    compute_dt(g, st, cfl, dt);
    free(st);
}

/* ------------------------------------------------------------------------------------------------ */
/* refinement criterion (the grid adapts between steps on the CPU, Sec. 2-3; the paper gives no       */
/* criterion: reading)                                                                              */
/*                                                                                                  */
/* Per block: the largest normalised jump, over its cells and the three axes, of the density and of  */
/* the squared field strength between the two face neighbours of a cell (ghost cells included):      */
/*   ind = max over cells, axes d, q in {rho, |B|^2} of |q(c + e_d) - q(c - e_d)| / (q(c + e_d) +    */
/*   q(c - e_d) + 1e-300).                                                                          */
/* A level-0 root whose indicator reaches r_refine is refined into its 8 children; a refined root    */
/* whose 8 children all stay below r_coarsen (< r_refine) is coarsened into it; other roots keep    */
/* their blocks. The new block list runs over each simulation's roots with x fastest, a refined root  */
/* listing its children with x fastest. Two levels only, so the result is always 2:1 balanced.       */

void or_block_indicator(const or_grid *g, const double *U, double *ind)
{
    double *st = pad_alloc(g->nb);
    pad_from_ext(g, U, st);
    exchange_messages(g, st);
    for (int b = 0; b < g->nb; b++) {
        double m = 0.0;
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++)
                    for (int d = 0; d < 3; d++) {
                        int p[3] = {i, j, k}, q[3] = {i, j, k};
                        p[d] += 1;
                        q[d] -= 1;
                        const double *cp = pcell(st, b, p[0], p[1], p[2]), *cm = pcell(st, b, q[0], q[1], q[2]);
                        double rp = cp[0], rm = cm[0];
                        double bp = cp[4] * cp[4] + cp[5] * cp[5] + cp[6] * cp[6];
                        double bm = cm[4] * cm[4] + cm[5] * cm[5] + cm[6] * cm[6];
                        double jr = fabs(rp - rm) / (rp + rm + 1e-300);
                        double jb = fabs(bp - bm) / (bp + bm + 1e-300);
                        if (jr > m) m = jr;
                        if (jb > m) m = jb;
                    }
        ind[b] = m;
    }
    free(st);
}

/* The adapted block list (levels, block indices, simulations) for indicators ind[nB]; returns the
 * number of blocks, or -1 when out_cap is too small. */
long or_adapt(const or_grid *g, const double *ind, double r_refine, double r_coarsen, int32_t *out_level,
              int32_t *out_ijk, int32_t *out_sim, long out_cap)
{
    long n = 0;
    for (int s = 0; s < g->ns; s++) {
        const or_sim *sm = &g->sims[s];
        for (long z = 0; z < sm->nroot[2]; z++)
            for (long y = 0; y < sm->nroot[1]; y++)
                for (long x = 0; x < sm->nroot[0]; x++) {
                    long r[3] = {x, y, z};
                    int root = lut_get(g, s, 0, r);
                    int refine;
                    if (root >= 0) {
                        refine = ind[root] >= r_refine;
                    } else {
                        double m = 0.0;
                        for (int q = 0; q < 8; q++) {
                            long c[3] = {2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2)};
                            double v = ind[lut_get(g, s, 1, c)];
                            if (v > m) m = v;
                        }
                        refine = !(m < r_coarsen);
                    }
                    if (n + (refine ? 8 : 1) > out_cap) return -1;
                    if (!refine) {
                        out_level[n] = 0;
                        for (int a = 0; a < 3; a++) out_ijk[3 * n + a] = (int32_t)r[a];
                        out_sim[n++] = s;
                    } else {
                        for (int q = 0; q < 8; q++) {
                            out_level[n] = 1;
                            out_ijk[3 * n + 0] = (int32_t)(2 * x + (q & 1));
                            out_ijk[3 * n + 1] = (int32_t)(2 * y + ((q >> 1) & 1));
                            out_ijk[3 * n + 2] = (int32_t)(2 * z + (q >> 2));
                            out_sim[n++] = s;
                        }
                    }
                }
    }
    return n;
}

/* Move a state to another grid of the same simulations after a refinement change (Sec. 2: a block is
 * refined into its 8 children, or 8 children are coarsened into their parent; Sec. 3 does this on the CPU
 * between steps, then rebuilds the message maps). Every cell of `to` takes the value the ghost rules of
 * `from` give at its level and global index: the leaf's own value where the block is unchanged, the
 * prolongation of a fine ghost cell (parent value plus limited slopes) where a level-0 block was refined,
 * the restriction (pairwise-tree mean) where 8 level-1 blocks were coarsened. Returns -1 when the
 * simulations differ or `to` holds a block that `from` cannot supply this way. */
static int same_sim(const or_sim *a, const or_sim *b)
{
    for (int q = 0; q < 3; q++)
        if (a->nroot[q] != b->nroot[q] || a->origin[q] != b->origin[q] || a->body_c[q] != b->body_c[q]) return 0;
    for (int q = 0; q < 6; q++)
        if (a->bc[q] != b->bc[q]) return 0;
    for (int q = 0; q < NV; q++)
        if (a->inflow_w[q] != b->inflow_w[q]) return 0;
    return a->dx0 == b->dx0 && a->body_r == b->body_r;
}

int or_remap(const or_grid *from, const double *U_from, const or_grid *to, double *U_to)
{
    if (from->ns != to->ns) return -1;
    for (int s = 0; s < from->ns; s++)
        if (!same_sim(&from->sims[s], &to->sims[s])) return -1;
    for (int b = 0; b < to->nb; b++) {
        int s = to->sim[b], l = to->level[b];
        long bb[3] = {to->ijk[3 * b], to->ijk[3 * b + 1], to->ijk[3 * b + 2]};
        int ok = lut_get(from, s, l, bb) >= 0;
        if (!ok && l == 1) {
            long pb[3] = {bb[0] / 2, bb[1] / 2, bb[2] / 2};
            ok = lut_get(from, s, 0, pb) >= 0;
        }
        if (!ok && l == 0) {
            ok = 1;
            for (int q = 0; q < 8; q++) {
                long cb[3] = {2 * bb[0] + (q & 1), 2 * bb[1] + ((q >> 1) & 1), 2 * bb[2] + ((q >> 2) & 1)};
                if (lut_get(from, s, 1, cb) < 0) ok = 0;
            }
        }
        if (!ok) return -1;
    }
    double *st = pad_alloc(from->nb);
    pad_from_ext(from, U_from, st);
    const size_t nbp = (size_t)to->nb * NC * NC * NC;
    for (int b = 0; b < to->nb; b++) {
        int s = to->sim[b], l = to->level[b];
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    long G[3] = {(long)to->ijk[3 * b] * NC + i, (long)to->ijk[3 * b + 1] * NC + j,
                                 (long)to->ijk[3 * b + 2] * NC + k};
                    double u[NV];
                    ghost_value(from, st, s, l, G, u);
                    for (int v = 0; v < NV; v++) U_to[v * nbp + (size_t)b * NC * NC * NC + (k * NC + j) * NC + i] = u[v];
                }
    }
    free(st);
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* message passing between processes (Sec. 4.2-4.4, Algorithms 3 and 4), with the processes simulated */
/* in one address space                                                                             */
/*                                                                                                  */
/* Blocks are assigned to processes (rank[b]); a process holds its blocks in its own padded array,   */
/* in ascending order of global block id (the local index). Ghost cells come from messages: a copy   */
/* from an equal-level neighbour, a restriction computed by a finer sender, or a prolongation         */
/* computed by a coarser sender. Messages between blocks of one process are copied directly ("local  */
/* message passing"); others go through one buffer per (sender, receiver) pair. Copies and            */
/* restrictions travel first (pass 1); prolongations (pass 2) are computed from the sender's ghost    */
/* cells as they stand after pass 1. Ghost cells outside the domain are filled by the receiver from  */
/* its own array (outflow, inflow) after the passes that feed them.                                  */
/*                                                                                                  */
/* A message from sender block b: its direction slot is dir * 4 + sub, dir the direction index of    */
/* the neighbour table (dx fastest) and sub the finer neighbour's position (0 otherwise); its          */
/* receive box is the part of the receiver's padded box [-2, 10)^3 covered by b's cells at the        */
/* receiver's level. The counting loop runs over the process's blocks in local order and the slots in */
/* ascending order; message i_M to a peer starts at start(i_M) = start(i_M - 1) + n_C + n_V *         */
/* cells(i_M - 1), n_C = 1 + 2 n_D = 7 header values (receiving block's local index on the peer, the   */
/* box's low corner, its high corner, inclusive) followed by the values in the order (v, i, j, k),    */
/* v fastest. A slot that would repeat a receiver placement already sent from b is skipped.           */

enum { MSG_COPY = 0, MSG_RESTRICT = 1, MSG_PROLONG = 2 };
#define XCHG_NC 7

typedef struct {
    int sender, receiver; /* global block ids */
    int type, pass, slot;
    int lo[3], hi[3];     /* receive box in the receiver's padded coordinates, inclusive */
    long ru[3];           /* the receiver's block position at its level, unwrapped as seen from the sender */
} or_msg;

static long floordiv(long a, long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

/* All messages sent by block b, in slot order; returns their count (at most 26 * 4). */
static int block_messages(const or_grid *g, int b, or_msg *out)
{
    int s = g->sim[b], l = g->level[b];
    const or_sim *sm = &g->sims[s];
    int n = 0, dn = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                int dir = dn++;
                int dd[3] = {dx, dy, dz};
                long p[3], pw[3];
                int inside = 1;
                for (int a = 0; a < 3; a++) {
                    long N = nblk_axis(sm, l, a);
                    p[a] = (long)g->ijk[3 * b + a] + dd[a];
                    pw[a] = p[a];
                    if (p[a] < 0 || p[a] >= N) {
                        if (sm->bc[2 * a + (p[a] < 0 ? 0 : 1)] != BC_PERIODIC) inside = 0;
                        pw[a] = (p[a] + N) % N;
                    }
                }
                if (!inside) continue;
                or_msg cand[4];
                int nc = 0;
                int id = lut_get(g, s, l, pw);
                if (id >= 0) { /* equal level */
                    cand[0].receiver = id;
                    cand[0].type = MSG_COPY;
                    for (int a = 0; a < 3; a++) cand[0].ru[a] = p[a];
                    nc = 1;
                } else if (l == 1) { /* the region is coarser: restriction to the level-0 block there */
                    long cu[3], cw[3];
                    for (int a = 0; a < 3; a++) {
                        cu[a] = floordiv(p[a], 2);
                        long N = nblk_axis(sm, 0, a);
                        cw[a] = ((cu[a] % N) + N) % N;
                    }
                    cand[0].receiver = lut_get(g, s, 0, cw);
                    cand[0].type = MSG_RESTRICT;
                    for (int a = 0; a < 3; a++) cand[0].ru[a] = cu[a];
                    nc = 1;
                } else { /* the region is finer: prolongation to each finer block touching b */
                    int m = 0;
                    for (int sz = 0; sz < 2; sz++)
                        for (int sy = 0; sy < 2; sy++)
                            for (int sx = 0; sx < 2; sx++) {
                                int sub[3] = {sx, sy, sz}, ok = 1;
                                for (int a = 0; a < 3; a++) {
                                    if (dd[a] == 1 && sub[a] != 0) ok = 0;
                                    if (dd[a] == -1 && sub[a] != 1) ok = 0;
                                }
                                if (!ok) continue;
                                long fw[3];
                                for (int a = 0; a < 3; a++) fw[a] = 2 * pw[a] + sub[a];
                                cand[nc].receiver = lut_get(g, s, 1, fw);
                                cand[nc].type = MSG_PROLONG;
                                for (int a = 0; a < 3; a++) cand[nc].ru[a] = 2 * p[a] + sub[a];
                                cand[nc].slot = m++;
                                nc++;
                            }
                }
                for (int c = 0; c < nc; c++) {
                    or_msg *mm = &cand[c];
                    int sub = mm->type == MSG_PROLONG ? mm->slot : 0;
                    int rl = g->level[mm->receiver];
                    /* b's cells at the receiver's level, relative to the receiver's origin */
                    long scale_num = rl > l ? 2 : 1, scale_den = rl < l ? 2 : 1;
                    int empty = 0;
                    for (int a = 0; a < 3; a++) {
                        long lo = (long)g->ijk[3 * b + a] * 8 * scale_num / scale_den - 8 * mm->ru[a];
                        long hi = lo + 8 * scale_num / scale_den;
                        if (lo < -2) lo = -2;
                        if (hi > 10) hi = 10;
                        if (lo >= hi) empty = 1;
                        mm->lo[a] = (int)lo;
                        mm->hi[a] = (int)hi - 1;
                    }
                    if (empty) continue;
                    int dup = 0;
                    for (int q = 0; q < n; q++)
                        if (out[q].receiver == mm->receiver && out[q].ru[0] == mm->ru[0] && out[q].ru[1] == mm->ru[1] &&
                            out[q].ru[2] == mm->ru[2])
                            dup = 1;
                    if (dup) continue;
                    mm->sender = b;
                    mm->pass = mm->type == MSG_PROLONG ? 2 : 1;
                    mm->slot = dir * 4 + sub;
                    out[n++] = *mm;
                }
            }
    return n;
}

static long box_cells(const or_msg *m)
{
    return (long)(m->hi[0] - m->lo[0] + 1) * (m->hi[1] - m->lo[1] + 1) * (m->hi[2] - m->lo[2] + 1);
}

/* The value of receive cell (i, j, k) of message m, from the sender's padded array sb (block m->sender's
 * cells at their process-local slot). */
static void message_value(const or_grid *g, const or_msg *m, const double *sst, int sb, int i, int j, int k,
                          double *u)
{
    int b = m->sender, sl = g->level[b];
    long gr[3] = {8 * m->ru[0] + i, 8 * m->ru[1] + j, 8 * m->ru[2] + k}; /* receiver level, unwrapped */
    if (m->type == MSG_COPY) {
        memcpy(u, pcell((double *)sst, sb, (int)(gr[0] - 8L * g->ijk[3 * b]), (int)(gr[1] - 8L * g->ijk[3 * b + 1]),
                        (int)(gr[2] - 8L * g->ijk[3 * b + 2])),
               sizeof(double) * NV);
    } else if (m->type == MSG_RESTRICT) {
        double c[8][NV];
        for (int q = 0; q < 8; q++) {
            long f[3] = {2 * gr[0] + (q & 1), 2 * gr[1] + ((q >> 1) & 1), 2 * gr[2] + ((q >> 2) & 1)};
            memcpy(c[q], pcell((double *)sst, sb, (int)(f[0] - 8L * g->ijk[3 * b]), (int)(f[1] - 8L * g->ijk[3 * b + 1]),
                               (int)(f[2] - 8L * g->ijk[3 * b + 2])),
                   sizeof(double) * NV);
        }
        for (int v = 0; v < NV; v++) {
            double cv[8];
            for (int q = 0; q < 8; q++) cv[q] = c[q][v];
            u[v] = or_restrict8(cv);
        }
    } else {
        long C[3];
        int sg[3];
        for (int a = 0; a < 3; a++) {
            C[a] = floordiv(gr[a], 2) - 8L * g->ijk[3 * b + a];
            sg[a] = (gr[a] & 1) ? 1 : -1;
        }
        (void)sl;
        const double *uc = pcell((double *)sst, sb, (int)C[0], (int)C[1], (int)C[2]);
        const double *um[3], *up[3];
        for (int d = 0; d < 3; d++) {
            long cm[3] = {C[0], C[1], C[2]}, cp[3] = {C[0], C[1], C[2]};
            cm[d] -= 1;
            cp[d] += 1;
            um[d] = pcell((double *)sst, sb, (int)cm[0], (int)cm[1], (int)cm[2]);
            up[d] = pcell((double *)sst, sb, (int)cp[0], (int)cp[1], (int)cp[2]);
        }
        for (int v = 0; v < NV; v++) {
            double cm[3] = {um[0][v], um[1][v], um[2][v]}, cp[3] = {up[0][v], up[1][v], up[2][v]};
            u[v] = or_prolong1(uc[v], cm, cp, sg);
        }
    }
}

/* Ghost cells of block b outside the domain, from its own padded array: inflow when an out-of-domain
 * axis is an inflow face, otherwise the cell at the out-of-domain outflow axes clamped to the block's
 * boundary row (periodic axes keep their ghost index: those ghost cells came by message). */
static void fill_boundary_ghosts(const or_grid *g, int b, double *st, int lb)
{
    int s = g->sim[b], l = g->level[b];
    const or_sim *sm = &g->sims[s];
    for (int k = -NGH; k < NC + NGH; k++)
        for (int j = -NGH; j < NC + NGH; j++)
            for (int i = -NGH; i < NC + NGH; i++) {
                int ii[3] = {i, j, k}, src[3] = {i, j, k};
                int out = 0, inflow = 0;
                for (int a = 0; a < 3; a++) {
                    long G = (long)g->ijk[3 * b + a] * NC + ii[a];
                    long N = ncell_axis(sm, l, a);
                    if (G >= 0 && G < N) continue;
                    int t = sm->bc[2 * a + (G < 0 ? 0 : 1)];
                    if (t == BC_PERIODIC) continue;
                    out = 1;
                    if (t == BC_INFLOW) inflow = 1;
                    src[a] = G < 0 ? 0 : NC - 1;
                }
                if (!out) continue;
                double *c = pcell(st, lb, i, j, k);
                if (inflow) inflow_cons(g, s, c);
                else memcpy(c, pcell(st, lb, src[0], src[1], src[2]), sizeof(double) * NV);
            }
}

/* Every message of the grid for a block-to-process assignment, in the order of the counting loops:
 * sender process, pass, receiving process, then the sender's local block order and slot order.
 * Row q of out (16 values): sender process, receiving process, pass, i_M (index among the messages from
 * that sender to that receiver in that pass), start offset, sender block, slot, receiving block (global),
 * its local index on the receiving process, type (0 copy, 1 restriction, 2 prolongation), lo[3], hi[3].
 * Returns the number of messages, or -1 when out has fewer than max_rows rows. */
long or_xchg_messages(const or_grid *g, const int32_t *rank, int n_ranks, int64_t *out, long max_rows)
{
    int *local = malloc(sizeof(int) * (size_t)g->nb);
    int *count = calloc((size_t)n_ranks, sizeof(int));
    for (int b = 0; b < g->nb; b++) local[b] = count[rank[b]]++;
    or_msg *mb = malloc(sizeof(or_msg) * 26 * 4);
    long q = 0;
    for (int sp = 0; sp < n_ranks; sp++)
        for (int pass = 1; pass <= 2; pass++)
            for (int rp = 0; rp < n_ranks; rp++) {
                long im = 0, start = 0;
                for (int b = 0; b < g->nb; b++) {
                    if (rank[b] != sp) continue;
                    int nm = block_messages(g, b, mb);
                    for (int c = 0; c < nm; c++) {
                        const or_msg *m = &mb[c];
                        if (m->pass != pass || rank[m->receiver] != rp) continue;
                        if (q >= max_rows) {
                            free(mb); free(count); free(local);
                            return -1;
                        }
                        int64_t *r = out + q * 16;
                        r[0] = sp; r[1] = rp; r[2] = pass; r[3] = im; r[4] = start;
                        r[5] = b; r[6] = m->slot; r[7] = m->receiver; r[8] = local[m->receiver]; r[9] = m->type;
                        for (int a = 0; a < 3; a++) { r[10 + a] = m->lo[a]; r[13 + a] = m->hi[a]; }
                        start += XCHG_NC + NV * box_cells(m);
                        im++;
                        q++;
                    }
                }
            }
    free(mb);
    free(count);
    free(local);
    return q;
}

/* The exchange of Algorithm 4 over simulated processes: every process copies its blocks' interior
 * cells into its own padded array, then for pass 1 and pass 2 packs its messages (local ones straight
 * into its own array, the others into one buffer per receiving process at the counted start offsets,
 * each message a header and its values), the buffers move to their receivers, and every receiver unpacks
 * its buffers by reading each message's header; after pass 1 the level-0 blocks, after pass 2 the
 * level-1 blocks fill their ghost cells outside the domain. The result, every process's padded array
 * gathered back into global block order, is written to view[8][nB][12][12][12] (like or_fill_ghosts). */
int or_xchg_run(const or_grid *g, const int32_t *rank, int n_ranks, const double *U, double *view)
{
    int *local = malloc(sizeof(int) * (size_t)g->nb);
    int *count = calloc((size_t)n_ranks, sizeof(int));
    for (int b = 0; b < g->nb; b++) local[b] = count[rank[b]]++;
    double **st = malloc(sizeof(double *) * (size_t)n_ranks);
    for (int r = 0; r < n_ranks; r++) st[r] = pad_alloc(count[r] > 0 ? count[r] : 1);
    /* interiors */
    size_t nbc = (size_t)g->nb * 512;
    for (int b = 0; b < g->nb; b++)
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    double *c = pcell(st[rank[b]], local[b], i, j, k);
                    for (int v = 0; v < NV; v++) c[v] = U[v * nbc + (size_t)b * 512 + (k * 8 + j) * 8 + i];
                }
    or_msg *mb = malloc(sizeof(or_msg) * 26 * 4);
    for (int pass = 1; pass <= 2; pass++) {
        /* pack: buffers[sender][receiver] */
        double **buf = calloc((size_t)n_ranks * n_ranks, sizeof(double *));
        long *len = calloc((size_t)n_ranks * n_ranks, sizeof(long));
        for (int sp = 0; sp < n_ranks; sp++)
            for (int rp = 0; rp < n_ranks; rp++) {
                if (rp == sp) continue;
                /* counting loop: the sizes and start offsets of the messages from sp to rp */
                long total = 0;
                for (int b = 0; b < g->nb; b++) {
                    if (rank[b] != sp) continue;
                    int nm = block_messages(g, b, mb);
                    for (int c = 0; c < nm; c++)
                        if (mb[c].pass == pass && rank[mb[c].receiver] == rp) total += XCHG_NC + NV * box_cells(&mb[c]);
                }
                len[sp * n_ranks + rp] = total;
                buf[sp * n_ranks + rp] = malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
                long start = 0;
                for (int b = 0; b < g->nb; b++) {
                    if (rank[b] != sp) continue;
                    int nm = block_messages(g, b, mb);
                    for (int c = 0; c < nm; c++) {
                        const or_msg *m = &mb[c];
                        if (m->pass != pass || rank[m->receiver] != rp) continue;
                        double *h = buf[sp * n_ranks + rp] + start;
                        h[0] = local[m->receiver];
                        for (int a = 0; a < 3; a++) { h[1 + a] = m->lo[a]; h[4 + a] = m->hi[a]; }
                        double *d = h + XCHG_NC;
                        for (int k = m->lo[2]; k <= m->hi[2]; k++)
                            for (int j = m->lo[1]; j <= m->hi[1]; j++)
                                for (int i = m->lo[0]; i <= m->hi[0]; i++) {
                                    message_value(g, m, st[sp], local[b], i, j, k, d);
                                    d += NV;
                                }
                        start += XCHG_NC + NV * box_cells(m);
                    }
                }
            }
        /* local message passing */
        for (int b = 0; b < g->nb; b++) {
            int nm = block_messages(g, b, mb);
            for (int c = 0; c < nm; c++) {
                const or_msg *m = &mb[c];
                if (m->pass != pass || rank[m->receiver] != rank[b]) continue;
                for (int k = m->lo[2]; k <= m->hi[2]; k++)
                    for (int j = m->lo[1]; j <= m->hi[1]; j++)
                        for (int i = m->lo[0]; i <= m->hi[0]; i++)
                            message_value(g, m, st[rank[b]], local[b], i, j, k,
                                          pcell(st[rank[b]], local[m->receiver], i, j, k));
            }
        }
        /* exchange and unpack: each receiver walks the buffer of each sender, message by message */
        for (int rp = 0; rp < n_ranks; rp++)
            for (int sp = 0; sp < n_ranks; sp++) {
                if (sp == rp) continue;
                const double *rb = buf[sp * n_ranks + rp];
                long at = 0, total = len[sp * n_ranks + rp];
                while (at < total) {
                    const double *h = rb + at;
                    int lb = (int)h[0], lo[3], hi[3];
                    for (int a = 0; a < 3; a++) { lo[a] = (int)h[1 + a]; hi[a] = (int)h[4 + a]; }
                    const double *d = h + XCHG_NC;
                    for (int k = lo[2]; k <= hi[2]; k++)
                        for (int j = lo[1]; j <= hi[1]; j++)
                            for (int i = lo[0]; i <= hi[0]; i++) {
                                memcpy(pcell(st[rp], lb, i, j, k), d, sizeof(double) * NV);
                                d += NV;
                            }
                    at = d - rb;
                }
            }
        for (int q = 0; q < n_ranks * n_ranks; q++) free(buf[q]);
        free(buf);
        free(len);
        /* ghost cells outside the domain */
        for (int b = 0; b < g->nb; b++)
            if (g->level[b] == pass - 1) fill_boundary_ghosts(g, b, st[rank[b]], local[b]);
    }
    size_t nbp = (size_t)g->nb * NPAD;
    for (int b = 0; b < g->nb; b++)
        for (size_t c = 0; c < NPAD; c++)
            for (int v = 0; v < NV; v++)
                view[v * nbp + (size_t)b * NPAD + c] = st[rank[b]][((size_t)local[b] * NPAD + c) * NV + v];
    free(mb);
    for (int r = 0; r < n_ranks; r++) free(st[r]);
    free(st);
    free(count);
    free(local);
    return 0;
}

/* Count of fluid cells whose density or pressure is not positive (or not finite). */
static long count_faults(const or_grid *g, double *st)
{
    long n = 0;
    for (int b = 0; b < g->nb; b++)
        for (int k = 0; k < NC; k++)
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    if (is_body(g, b, i, j, k)) continue;
                    double w[NV];
                    or_cons_to_prim(pcell(st, b, i, j, k), w);
                    if (!(w[0] > 0.0) || !(w[7] > 0.0)) n++;
                }
    return n;
}

/* ------------------------------------------------------------------------------------------------ */
/* learned flux correction (the learned form; not in the paper)                                      */
/*                                                                                                  */
/* Face order of one block: face f of axis d lies between cells f-1 and f along d; its index is     */
/* (t2 * 8 + t1) * 9 + f for d = 0 (t1 = y, t2 = z), (t2 * 9 + f) * 8 + t1 for d = 1 (t1 = x, t2 = z)   */
/* and (f * 8 + t2) * 8 + t1 for d = 2 (t1 = x, t2 = y); globally (b * 3 + d) * 576 + index. Faces on a */
/* block face appear once per block that owns them.                                                 */
/* Face-normal frame of axis d: (rho, u_n, u_t1, u_t2, B_n, B_t1, B_t2, p) with (n, t1, t2) = (d,     */
/* d + 1, d + 2) taken cyclically (x -> y -> z -> x); fluxes likewise with the momentum and field      */
/* components.                                                                                      */

static int face_slot(int d, int f, int t1, int t2)
{
    if (d == 0) return (t2 * 8 + t1) * 9 + f;
    if (d == 1) return (t2 * 9 + f) * 8 + t1;
    return (f * 8 + t2) * 8 + t1;
}

/* Stencil features of every face: the primitives of the 4 cells f-2 .. f+1 along d, each in the
 * face-normal frame, z-scored with stats (mean[32], std[32]) when stats is not NULL:
 * X[(b * 3 + d) * 576 + slot][q * 8 + v] = (w_q,v - mean[q * 8 + v]) / std[q * 8 + v]. */
void or_face_features(const or_grid *g, const double *U, const double *stats, double *X)
{
    double *st = pad_alloc(g->nb);
    pad_from_ext(g, U, st);
    exchange_messages(g, st);
    for (int b = 0; b < g->nb; b++)
        for (int d = 0; d < 3; d++)
            for (int t2 = 0; t2 < NC; t2++)
                for (int t1 = 0; t1 < NC; t1++)
                    for (int f = 0; f <= NC; f++) {
                        double *x = X + ((size_t)(b * 3 + d) * 576 + (size_t)face_slot(d, f, t1, t2)) * 32;
                        for (int q = 0; q < 4; q++) {
                            int c[3];
                            face_cell(d, f - 2 + q, t1, t2, c);
                            double w[NV], r[NV];
                            or_cons_to_prim(pcell(st, b, c[0], c[1], c[2]), w);
                            r[0] = w[0];
                            r[7] = w[7];
                            for (int a = 0; a < 3; a++) {
                                r[1 + a] = w[1 + (d + a) % 3];
                                r[4 + a] = w[4 + (d + a) % 3];
                            }
                            for (int v = 0; v < NV; v++) {
                                int e = q * 8 + v;
                                x[e] = stats ? (r[v] - stats[e]) / stats[32 + e] : r[v];
                            }
                        }
                    }
    free(st);
}

/* The flag of the cell on the other side of face (d, side) of cell (i, j, k) of block b on a
 * single-level grid: 0 when that side is outside the domain through a non-periodic face. */
static int other_side_flag(const or_grid *g, const unsigned char *flags, int b, const int ii[3], int d, int side)
{
    int s = g->sim[b];
    const or_sim *sm = &g->sims[s];
    long G[3];
    for (int a = 0; a < 3; a++) G[a] = (long)g->ijk[3 * b + a] * NC + ii[a];
    G[d] += side ? 1 : -1;
    long N = ncell_axis(sm, 0, d);
    if (G[d] < 0 || G[d] >= N) {
        if (sm->bc[2 * d + (G[d] < 0 ? 0 : 1)] != BC_PERIODIC) return 0;
        G[d] = (G[d] + N) % N;
    }
    long bb[3] = {G[0] / NC, G[1] / NC, G[2] / NC};
    int nb = lut_get(g, s, 0, bb);
    return flags[(size_t)nb * 512 + ((G[2] % NC) * NC + G[1] % NC) * NC + G[0] % NC];
}

/* Advance n_stages stages with the learned correction. y[(b * 3 + d) * 576 + slot][8]: the normalised
 * flux correction of every face in the face-normal frame, the same for every stage; ystats: out_mean[8],
 * out_std[8]. Per stage:
 *   1. ghost exchange and the plain fluxes F (as or_advance);
 *   2. dF = y * out_std + out_mean, rotated from the face-normal frame to x, y, z; F' = F + dF, except on
 *      faces next to a body cell (those keep F);
 *   3. a provisional update with F';
 *   4. a fluid cell is flagged when its provisional rho <= 0 or p <= 0, or its provisional rho (p) leaves
 *      [lo - tau h, hi + tau h], where lo and hi are the minimum and maximum of rho (p) over the cell and
 *      its six face neighbours in the stage input and h = max(hi - lo, floor_rel * max(|lo|, |hi|))
 *      (floor_rel = 0: h is the range);
 *   5. every face with a flagged cell on either side takes F again, for both cells, and the stage is
 *      recomputed once from these fluxes (no second test).
 * Single-level grids only (returns -1 otherwise). *flagged accumulates the flagged cells of all stages;
 * *faults counts non-positive cells after the last stage. */
int or_advance_learned(const or_grid *g, double *U0, double *U1, double *dt, int n_stages, const or_opts *o,
                       const double *y, const double *ystats, double tau, double floor_rel, long *faults,
                       long *flagged)
{
    if (o->n_table != 2 || o->local_dt) return -1;
    for (int b = 0; b < g->nb; b++)
        if (g->level[b] != 0 || has_level_change(g, b)) return -1;
    double *s0 = pad_alloc(g->nb), *s1 = pad_alloc(g->nb);
    pad_from_ext(g, U0, s0);
    pad_from_ext(g, U1, s1);
    or_faces *plain = malloc(sizeof(or_faces) * (size_t)g->nb);
    or_faces *used = malloc(sizeof(or_faces) * (size_t)g->nb);
    unsigned char *flags = calloc((size_t)g->nb * 512, 1);
    long nflag = 0;
    for (int st = 0; st < n_stages; st++) {
        int e = st % 2;
        double alpha = o->alpha[e], beta = o->beta[e];
        double *in = e ? s1 : s0, *out = e ? s0 : s1;
        if (e == 0 && o->recompute_dt) compute_dt(g, s0, o->cfl, dt);
        exchange_messages(g, in);
        /* the second stage writes over U^n, which the recompute of step 5 reads again: keep a copy */
        double *u0 = s0;
        if (e == 1) {
            u0 = pad_alloc(g->nb);
            memcpy(u0, s0, sizeof(double) * (size_t)g->nb * NPAD * NV);
        }
        /* steps 1-3 */
        for (int b = 0; b < g->nb; b++) {
            calc_face_values_and_fluxes(g, b, in, o, &plain[b]);
            memcpy(&used[b], &plain[b], sizeof(or_faces));
            for (int d = 0; d < 3; d++)
                for (int t2 = 0; t2 < NC; t2++)
                    for (int t1 = 0; t1 < NC; t1++)
                        for (int f = 0; f <= NC; f++) {
                            int cl[3], cr[3];
                            face_cell(d, f - 1, t1, t2, cl);
                            face_cell(d, f, t1, t2, cr);
                            if (is_body(g, b, cl[0], cl[1], cl[2]) || is_body(g, b, cr[0], cr[1], cr[2])) continue;
                            const double *yf = y + ((size_t)(b * 3 + d) * 576 + (size_t)face_slot(d, f, t1, t2)) * 8;
                            double dn[NV], dF[NV];
                            for (int v = 0; v < NV; v++) dn[v] = yf[v] * ystats[8 + v] + ystats[v];
                            dF[0] = dn[0];
                            dF[7] = dn[7];
                            for (int a = 0; a < 3; a++) {
                                dF[1 + (d + a) % 3] = dn[1 + a];
                                dF[4 + (d + a) % 3] = dn[4 + a];
                            }
                            double *fv = used[b].f[d][f][t2][t1];
                            for (int v = 0; v < NV; v++) fv[v] = fv[v] + dF[v];
                        }
            calc_source_and_update(g, b, in, u0, out, dt[g->sim[b]], NULL, alpha, beta, o, &used[b]);
        }
        /* step 4 */
        for (int b = 0; b < g->nb; b++)
            for (int k = 0; k < NC; k++)
                for (int j = 0; j < NC; j++)
                    for (int i = 0; i < NC; i++) {
                        unsigned char *fl = &flags[(size_t)b * 512 + (k * NC + j) * NC + i];
                        *fl = 0;
                        if (is_body(g, b, i, j, k)) continue;
                        double w[NV];
                        or_cons_to_prim(pcell(out, b, i, j, k), w);
                        const int nb7[7][3] = {{i, j, k}, {i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                                               {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
                        double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
                        for (int q = 0; q < 7; q++) {
                            double wo[NV];
                            or_cons_to_prim(pcell(in, b, nb7[q][0], nb7[q][1], nb7[q][2]), wo);
                            const double val[2] = {wo[0], wo[7]};
                            for (int m = 0; m < 2; m++) {
                                if (val[m] < lo[m]) lo[m] = val[m];
                                if (val[m] > hi[m]) hi[m] = val[m];
                            }
                        }
                        const double now[2] = {w[0], w[7]};
                        int bad = !(w[0] > 0.0) || !(w[7] > 0.0);
                        for (int m = 0; m < 2; m++) {
                            double h = hi[m] - lo[m];
                            double fh = floor_rel * fmax(fabs(lo[m]), fabs(hi[m]));
                            if (fh > h) h = fh;
                            if (now[m] < lo[m] - tau * h || now[m] > hi[m] + tau * h) bad = 1;
                        }
                        *fl = (unsigned char)bad;
                        nflag += bad;
                    }
        /* step 5 */
        for (int b = 0; b < g->nb; b++) {
            int any = 0;
            for (int d = 0; d < 3; d++)
                for (int t2 = 0; t2 < NC; t2++)
                    for (int t1 = 0; t1 < NC; t1++)
                        for (int f = 0; f <= NC; f++) {
                            int cl[3], cr[3];
                            face_cell(d, f - 1, t1, t2, cl);
                            face_cell(d, f, t1, t2, cr);
                            int fl_l = f > 0 ? flags[(size_t)b * 512 + (cl[2] * NC + cl[1]) * NC + cl[0]]
                                             : other_side_flag(g, flags, b, cr, d, 0);
                            int fl_r = f < NC ? flags[(size_t)b * 512 + (cr[2] * NC + cr[1]) * NC + cr[0]]
                                              : other_side_flag(g, flags, b, cl, d, 1);
                            if (!(fl_l || fl_r)) continue;
                            memcpy(used[b].f[d][f][t2][t1], plain[b].f[d][f][t2][t1], sizeof(double) * NV);
                            any = 1;
                        }
            if (any) calc_source_and_update(g, b, in, u0, out, dt[g->sim[b]], NULL, alpha, beta, o, &used[b]);
        }
        if (u0 != s0) free(u0);
    }
    if (faults) *faults = count_faults(g, (n_stages % 2) ? s1 : s0);
    if (flagged) *flagged = nflag;
    pad_to_ext(g, s0, U0);
    pad_to_ext(g, s1, U1);
    free(flags);
    free(used);
    free(plain);
    free(s0);
    free(s1);
    return 0;
}

/* Advance n_stages stages. Stage s uses table entry s % n_table; even stages read U0 and write U1,
 * odd stages read U1 (and U0 as the step's starting state) and overwrite U0. With recompute_dt, dt is
 * recomputed from U0 at the start of every step; otherwise dt[] is used as given. On return dt[] holds
 * the last step's dt and *faults the number of non-positive cells after the last stage. With local_dt,
 * dt[] holds one dt per cell ([nB][8][8][8], local time stepping) instead of one per simulation. */
int or_advance(const or_grid *g, double *U0, double *U1, double *dt, int n_stages, const or_opts *o, long *faults)
{
    if (o->n_table != 2) return -1;
    double *s0 = pad_alloc(g->nb), *s1 = pad_alloc(g->nb);
    pad_from_ext(g, U0, s0);
    pad_from_ext(g, U1, s1);
    or_faces **faces = calloc((size_t)g->nb, sizeof(or_faces *));
    int any_change = 0;
    for (int b = 0; b < g->nb; b++)
        if (has_level_change(g, b)) {
            faces[b] = malloc(sizeof(or_faces));
            any_change = 1;
        }
    for (int st = 0; st < n_stages; st++) {
        int e = st % 2;
        double alpha = o->alpha[e], beta = o->beta[e];
        double *in = e ? s1 : s0, *out = e ? s0 : s1;
        if (e == 0 && o->recompute_dt) {
            if (o->local_dt) compute_local_dt(g, s0, o->cfl, dt);
            else compute_dt(g, s0, o->cfl, dt);
        }
        exchange_messages(g, in);
#pragma omp parallel
        {
            or_faces *tmp = malloc(sizeof(or_faces));
#pragma omp for schedule(dynamic, 4)
            for (int b = 0; b < g->nb; b++) {
                or_faces *F = faces[b] ? faces[b] : tmp;
                calc_face_values_and_fluxes(g, b, in, o, F);
                const double *dloc = o->local_dt ? dt + (size_t)b * NC * NC * NC : NULL;
                calc_source_and_update(g, b, in, s0, out, o->local_dt ? 0.0 : dt[g->sim[b]], dloc, alpha, beta,
                                       o, F);
            }
            free(tmp);
        }
        if (any_change) flux_correction(g, faces, out, dt, o->local_dt, beta);
    }
    if (faults) *faults = count_faults(g, (n_stages % 2) ? s1 : s0);
    pad_to_ext(g, s0, U0);
    pad_to_ext(g, s1, U1);
    for (int b = 0; b < g->nb; b++) free(faces[b]);
    free(faces);
    free(s0);
    free(s1);
    return 0;
}
