/*
 * Plain FP64 CPU oracle for the MDLG hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the bench
 * may load this library.  It shares no code, header, table or helper with the
 * HIP path: it is written directly from the paper (Parsa & Wagner,
 * "Lattice Gas with Molecular Dynamics Collision Operator"), in the paper's
 * notation, scalar, unblocked and in double precision, so that a reader can
 * check it against the text by eye.
 *
 * What it computes, with the passage each part follows:
 *   - Lennard-Jones pair energy and force (section "MDLG for a two-dimensional
 *     Lennard-Jones gas", the LJ potential equation); the force is minus the
 *     gradient of the pair potential (section "Lattice Gas with Molecular
 *     Dynamics collision operator", Newton's equations).  Cut off at r_c with
 *     the energy shifted by V(r_c) (the paper runs LAMMPS and does not state
 *     cutoff or shift; this is the reading used throughout).
 *   - Velocity-Verlet integration in a periodic box with integer image
 *     counters (Newton's equations; the integrator is not stated in the paper).
 *   - MDLG binning: occupation numbers n_i(x,t) of eq. (MDni), the local
 *     particle number N(x,t), the lattice momentum N u = sum_i v_i n_i and the
 *     second moment sum_i v_i v_i n_i, accumulated per site over lattice steps
 *     (eq. (fieq): f_i^eq is the site and time average of n_i).
 *   - The continuous displacement delta x = x(t) - x(t - Delta t) used in
 *     eq. (eqn:a) for a^2, accumulated as sums of delta x and delta x^2.
 *
 * Readings where the paper is silent or ambiguous (all shared with the GPU
 * path by specification, not by code):
 *   - cell indicator: a particle belongs to site c along axis alpha when
 *     c*dx <= x_alpha < (c+1)*dx (floor), i.e. the half-open interval is
 *     closed below instead of above; the two differ on a set of measure zero.
 *   - periodic boundaries: positions are unwrapped with image counters before
 *     the lattice displacement v = C(t) - C(t - Delta t) is taken.
 *   - velocity window: lattice velocities with |v_alpha| <= V for every axis
 *     get a bin i = sum_alpha (v_alpha + V) (2V+1)^alpha; other particles are
 *     counted as overflow at their arrival site.  Density and moments include
 *     every particle, so sum_i n_i + overflow = N(x,t) exactly.
 *   - n_i(x,t) is indexed by the arrival site x at time t, as in eq. (MDni).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)

typedef struct {
    int dim;          /* 2 or 3 */
    int n;            /* number of particles */
    double box[3];    /* periodic box side per axis */
    double eps;       /* LJ interaction strength epsilon */
    double sigma;     /* LJ length sigma */
    double mass;      /* particle mass m */
    double rc;        /* cutoff radius */
    int forces_off;   /* 1: ideal gas, no forces */
    double dt;        /* MD time step */
} orc_md;

typedef struct {
    int M[3];         /* lattice sites per axis */
    double dx;        /* lattice spacing Delta x */
    int V;            /* velocity window half-width: |v_alpha| <= V */
} orc_lattice;

/* ------------------------------------------------------------------ */
/* Lennard-Jones pair interaction                                      */
/* ------------------------------------------------------------------ */

/* V(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] */
double orc_lj_potential(double r, double eps, double sigma)
{
    double sr = sigma / r;
    double sr6 = pow(sr, 6.0);
    return 4.0 * eps * (sr6 * sr6 - sr6);
}

/* Force on particle i from particle j, F_i = -dV/dx_i = g(r) (x_i - x_j),
 * with g(r) = -V'(r)/r = (24 eps / r^2) [2 (sigma/r)^12 - (sigma/r)^6].
 * Returns g(r). */
double orc_lj_force_over_r(double r, double eps, double sigma)
{
    double sr = sigma / r;
    double sr6 = pow(sr, 6.0);
    return 24.0 * eps / (r * r) * (2.0 * sr6 * sr6 - sr6);
}

/* minimum-image component of a difference along an axis of length L */
static double min_image(double d, double L)
{
    return d - L * nearbyint(d / L);
}

/* Accumulate the force of j on i (ordered pair) into acc[i], and half the
 * shifted pair energy into *epot. */
static void pair_accumulate(const orc_md *p, const double *x, int i, int j,
                            double *acc, double *epot, double vshift)
{
    int d = p->dim;
    double dr[3] = {0.0, 0.0, 0.0};
    double r2 = 0.0;
    for (int a = 0; a < d; ++a) {
        dr[a] = min_image(x[i * d + a] - x[j * d + a], p->box[a]);
        r2 += dr[a] * dr[a];
    }
    if (r2 >= p->rc * p->rc)
        return;
    double r = sqrt(r2);
    double g = orc_lj_force_over_r(r, p->eps, p->sigma);
    for (int a = 0; a < d; ++a)
        acc[i * d + a] += g * dr[a] / p->mass;
    if (epot)
        *epot += 0.5 * (orc_lj_potential(r, p->eps, p->sigma) - vshift);
}

/* Brute-force O(N^2) accelerations a_i = F_i / m over all ordered pairs with
 * minimum-image distance below r_c.  Potential energy (shifted) in *epot. */
int orc_forces_brute(const orc_md *p, const double *x, double *acc, double *epot)
{
    int d = p->dim, n = p->n;
    memset(acc, 0, sizeof(double) * (size_t)n * d);
    if (epot)
        *epot = 0.0;
    if (p->forces_off)
        return ORC_OK;
    double vshift = orc_lj_potential(p->rc, p->eps, p->sigma);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (j != i)
                pair_accumulate(p, x, i, j, acc, epot, vshift);
    return ORC_OK;
}

/* Plain linked-list cell grid of side >= r_c over all particles. */
typedef struct {
    int nc[3];
    int *head, *next, *cof;
} cell_grid;

static void free_grid(cell_grid *g)
{
    free(g->head);
    free(g->next);
    free(g->cof);
}

/* Returns 1 when an axis holds fewer than 3 cells (no grid), ORC_ENOMEM on
 * allocation failure, 0 with the grid built. */
static int build_grid(const orc_md *p, const double *x, cell_grid *g)
{
    int d = p->dim, n = p->n;
    double h[3] = {1.0, 1.0, 1.0};
    g->nc[0] = g->nc[1] = g->nc[2] = 1;
    g->head = g->next = g->cof = NULL;
    for (int a = 0; a < d; ++a) {
        g->nc[a] = (int)floor(p->box[a] / p->rc);
        if (g->nc[a] < 3)
            return 1;
        h[a] = p->box[a] / g->nc[a];
    }
    long ncell = (long)g->nc[0] * g->nc[1] * g->nc[2];
    g->head = (int *)malloc(sizeof(int) * ncell);
    g->next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    g->cof = (int *)malloc(sizeof(int) * 3 * (size_t)(n > 0 ? n : 1));
    if (!g->head || !g->next || !g->cof) {
        free_grid(g);
        return ORC_ENOMEM;
    }
    for (long c = 0; c < ncell; ++c)
        g->head[c] = -1;
    for (int i = 0; i < n; ++i) {
        int cc[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
            int q = (int)floor(x[i * d + a] / h[a]);
            if (q < 0) q = 0;
            if (q >= g->nc[a]) q = g->nc[a] - 1;
            cc[a] = q;
            g->cof[3 * i + a] = q;
        }
        long c = cc[0] + (long)g->nc[0] * (cc[1] + (long)g->nc[1] * cc[2]);
        g->next[i] = g->head[c];
        g->head[c] = i;
    }
    return 0;
}

/* Force on particle i from every j != i in its own and the neighbouring cells. */
static void cell_walk(const orc_md *p, const double *x, const cell_grid *g, int i, double *acc,
                      double *epot, double vshift)
{
    int d = p->dim;
    int span[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a)
        span[a] = 3;
    for (int oz = 0; oz < span[2]; ++oz)
        for (int oy = 0; oy < span[1]; ++oy)
            for (int ox = 0; ox < span[0]; ++ox) {
                int off[3] = {ox - 1, oy - 1, oz - 1};
                int cc[3] = {0, 0, 0};
                for (int a = 0; a < d; ++a)
                    cc[a] = ((g->cof[3 * i + a] + off[a]) % g->nc[a] + g->nc[a]) % g->nc[a];
                long c = cc[0] + (long)g->nc[0] * (cc[1] + (long)g->nc[1] * cc[2]);
                for (int j = g->head[c]; j >= 0; j = g->next[j])
                    if (j != i)
                        pair_accumulate(p, x, i, j, acc, epot, vshift);
            }
}

/* Same accelerations through a plain linked-list cell grid of side >= r_c.
 * Falls back to the brute-force sum when an axis holds fewer than 3 cells. */
int orc_forces_cells(const orc_md *p, const double *x, double *acc, double *epot)
{
    int d = p->dim, n = p->n;
    cell_grid g;
    int rc = build_grid(p, x, &g);
    if (rc == 1)
        return orc_forces_brute(p, x, acc, epot);
    if (rc != 0)
        return rc;
    memset(acc, 0, sizeof(double) * (size_t)n * d);
    if (epot)
        *epot = 0.0;
    if (!p->forces_off) {
        double vshift = orc_lj_potential(p->rc, p->eps, p->sigma);
        for (int i = 0; i < n; ++i)
            cell_walk(p, x, &g, i, acc, epot, vshift);
    }
    free_grid(&g);
    return ORC_OK;
}

/* Accelerations of the m particles idx[0..m) only (row k of acc_out for
 * particle idx[k]), each summed over all its partners exactly as above. */
int orc_forces_subset(const orc_md *p, const double *x, const int *idx, int m, double *acc_out)
{
    int d = p->dim, n = p->n;
    double *acc = (double *)calloc((size_t)(n > 0 ? n : 1) * d, sizeof(double));
    if (!acc)
        return ORC_ENOMEM;
    for (int k = 0; k < m; ++k)
        if (idx[k] < 0 || idx[k] >= n) {
            free(acc);
            return ORC_EINVAL;
        }
    if (!p->forces_off) {
        double vshift = orc_lj_potential(p->rc, p->eps, p->sigma);
        cell_grid g;
        int rc = build_grid(p, x, &g);
        if (rc == ORC_ENOMEM) {
            free(acc);
            return rc;
        }
        for (int k = 0; k < m; ++k) {
            int i = idx[k];
            for (int a = 0; a < d; ++a)
                acc[i * d + a] = 0.0;
            if (rc == 1) {
                for (int j = 0; j < n; ++j)
                    if (j != i)
                        pair_accumulate(p, x, i, j, acc, NULL, vshift);
            } else {
                cell_walk(p, x, &g, i, acc, NULL, vshift);
            }
        }
        if (rc == 0)
            free_grid(&g);
    }
    for (int k = 0; k < m; ++k)
        for (int a = 0; a < d; ++a)
            acc_out[k * d + a] = acc[idx[k] * d + a];
    free(acc);
    return ORC_OK;
}

/* Visit every ordered pair (i, j), i != j, within r_c (minimum image),
 * calling fn(ctx, i, j, r, r2) with r = x_i - x_j.  Uses a linked-list cell
 * grid of side >= r_c when every axis holds at least 3 cells, else all pairs. */
typedef void (*pair_fn)(void *ctx, int i, int j, const double *r, double r2);

static int visit_pairs(const orc_md *p, const double *x, pair_fn fn, void *ctx)
{
    int d = p->dim, n = p->n;
    int nc[3] = {1, 1, 1};
    double h[3] = {1.0, 1.0, 1.0};
    int cells = 1;
    for (int a = 0; a < d; ++a) {
        nc[a] = (int)floor(p->box[a] / p->rc);
        if (nc[a] < 3)
            cells = 0;
        else
            h[a] = p->box[a] / nc[a];
    }
    double rc2 = p->rc * p->rc;
    if (!cells) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                if (j == i)
                    continue;
                double r[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
                for (int a = 0; a < d; ++a) {
                    r[a] = min_image(x[i * d + a] - x[j * d + a], p->box[a]);
                    r2 += r[a] * r[a];
                }
                if (r2 < rc2)
                    fn(ctx, i, j, r, r2);
            }
        return ORC_OK;
    }
    for (int a = d; a < 3; ++a)
        nc[a] = 1;
    long ncell = (long)nc[0] * nc[1] * nc[2];
    int *head = (int *)malloc(sizeof(int) * ncell);
    int *next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *cof = (int *)malloc(sizeof(int) * 3 * (size_t)(n > 0 ? n : 1));
    if (!head || !next || !cof) {
        free(head); free(next); free(cof);
        return ORC_ENOMEM;
    }
    for (long c = 0; c < ncell; ++c)
        head[c] = -1;
    for (int i = 0; i < n; ++i) {
        int cc[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
            int q = (int)floor(x[i * d + a] / h[a]);
            if (q < 0) q = 0;
            if (q >= nc[a]) q = nc[a] - 1;
            cc[a] = q;
        }
        for (int a = 0; a < 3; ++a)
            cof[3 * i + a] = cc[a];
        long c = cc[0] + (long)nc[0] * (cc[1] + (long)nc[1] * cc[2]);
        next[i] = head[c];
        head[c] = i;
    }
    int span[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a)
        span[a] = 3;
    for (int i = 0; i < n; ++i)
        for (int oz = 0; oz < span[2]; ++oz)
            for (int oy = 0; oy < span[1]; ++oy)
                for (int ox = 0; ox < span[0]; ++ox) {
                    int off[3] = {ox - 1, oy - 1, oz - 1};
                    int cc[3] = {0, 0, 0};
                    for (int a = 0; a < d; ++a)
                        cc[a] = ((cof[3 * i + a] + off[a]) % nc[a] + nc[a]) % nc[a];
                    long c = cc[0] + (long)nc[0] * (cc[1] + (long)nc[1] * cc[2]);
                    for (int j = head[c]; j >= 0; j = next[j]) {
                        if (j == i)
                            continue;
                        double r[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
                        for (int a = 0; a < d; ++a) {
                            r[a] = min_image(x[i * d + a] - x[j * d + a], p->box[a]);
                            r2 += r[a] * r[a];
                        }
                        if (r2 < rc2)
                            fn(ctx, i, j, r, r2);
                    }
                }
    free(head);
    free(next);
    free(cof);
    return ORC_OK;
}

static int compute_forces(const orc_md *p, const double *x, double *acc,
                          double *epot, int use_cells)
{
    return use_cells ? orc_forces_cells(p, x, acc, epot)
                     : orc_forces_brute(p, x, acc, epot);
}

/* ------------------------------------------------------------------ */
/* Velocity Verlet with periodic wrap and image counters               */
/* ------------------------------------------------------------------ */

/* Bring a coordinate back into [0, L), moving the image counter along. */
static void wrap_coordinate(double *xa, int32_t *img, double L)
{
    while (*xa < 0.0) {
        *xa += L;
        *img -= 1;
    }
    while (*xa >= L) {
        *xa -= L;
        *img += 1;
    }
}

/* Rescale velocities so that sum m v^2 / (d (N - 1)) = kT. */
static void rescale_velocities(const orc_md *p, double *v, double kT)
{
    int d = p->dim, n = p->n;
    double s = 0.0;
    for (long k = 0; k < (long)n * d; ++k)
        s += p->mass * v[k] * v[k];
    if (s <= 0.0 || n < 2)
        return;
    double lam = sqrt(kT * d * (n - 1) / s);
    for (long k = 0; k < (long)n * d; ++k)
        v[k] *= lam;
}

/* Advance nsteps velocity-Verlet steps.  On entry acc must hold a(t) for the
 * positions x(t) (call orc_forces_* once first).  x is kept in [0, L) with the
 * image counters img carrying the number of box crossings.  When thermo_every
 * is positive, velocities are rescaled to kT after every step whose global
 * index (*step, counted from 1) is a multiple of thermo_every. */
int orc_vv(const orc_md *p, double *x, int32_t *img, double *v, double *acc,
           long nsteps, long *step, int thermo_every, double kT, int use_cells)
{
    int d = p->dim, n = p->n;
    long total = (long)n * d;
    for (long s = 0; s < nsteps; ++s) {
        for (long k = 0; k < total; ++k)
            v[k] += 0.5 * acc[k] * p->dt;
        for (long k = 0; k < total; ++k)
            x[k] += v[k] * p->dt;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < d; ++a)
                wrap_coordinate(&x[i * d + a], &img[i * d + a], p->box[a]);
        int rc = compute_forces(p, x, acc, NULL, use_cells);
        if (rc != ORC_OK)
            return rc;
        for (long k = 0; k < total; ++k)
            v[k] += 0.5 * acc[k] * p->dt;
        *step += 1;
        if (thermo_every > 0 && (*step % thermo_every) == 0)
            rescale_velocities(p, v, kT);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* MDLG binning (eq. MDni) and per-site moments                        */
/* ------------------------------------------------------------------ */

int orc_num_moments(int dim)
{
    /* N, overflow, sum v_alpha (dim), sum v_alpha v_beta (upper triangle) */
    return 2 + dim + dim * (dim + 1) / 2;
}

static long floor_to_long(double y)
{
    return (long)floor(y);
}

/* One lattice step: particles at unwrapped positions xu_prev (time t - Dt)
 * and xu_now (time t).  Adds n_i(x,t) to A[site][Q], and to mom[site][...]
 * the local number N(x,t), the overflow count, sum_i v_i n_i and
 * sum_i v_i v_i n_i (all particles), and to dsum/dsq the continuous
 * displacement sums.  Sites are x-fastest; bins are x-fastest in v + V. */
int orc_bin(const orc_lattice *L, int dim, int n, const double *xu_prev,
            const double *xu_now, uint64_t *A, int64_t *mom, double *dsum,
            double *dsq)
{
    if (dim < 2 || dim > 3 || L->V < 0)
        return ORC_EINVAL;
    int W = 2 * L->V + 1;
    int Q = 1;
    for (int a = 0; a < dim; ++a)
        Q *= W;
    int nm = orc_num_moments(dim);
    for (int j = 0; j < n; ++j) {
        long v[3] = {0, 0, 0};
        long site = 0, stride = 1;
        int inside = 1;
        long bin = 0, bstride = 1;
        for (int a = 0; a < dim; ++a) {
            long cnow = floor_to_long(xu_now[j * dim + a] / L->dx);
            long cprev = floor_to_long(xu_prev[j * dim + a] / L->dx);
            v[a] = cnow - cprev;
            long sa = ((cnow % L->M[a]) + L->M[a]) % L->M[a];
            site += sa * stride;
            stride *= L->M[a];
            if (v[a] < -L->V || v[a] > L->V)
                inside = 0;
            bin += (v[a] + L->V) * bstride;
            bstride *= W;
        }
        int64_t *m = mom + site * nm;
        m[0] += 1;
        if (inside)
            A[site * Q + bin] += 1;
        else
            m[1] += 1;
        for (int a = 0; a < dim; ++a)
            m[2 + a] += v[a];
        int k = 2 + dim;
        for (int a = 0; a < dim; ++a)
            for (int b = a; b < dim; ++b)
                m[k++] += v[a] * v[b];
        for (int a = 0; a < dim; ++a) {
            double dd = xu_now[j * dim + a] - xu_prev[j * dim + a];
            dsum[a] += dd;
            dsq[a] += dd * dd;
        }
    }
    return ORC_OK;
}

/* Literal evaluation of eq. (MDni) for tiny inputs: for every site x, every
 * window velocity v_i and every particle j, multiply the two cell indicators
 * Delta_x(x_j(t)) and Delta_{x - v_i}(x_j(t - Dt)), written as interval tests.
 * The periodic image of particle j at time t is removed from both positions
 * before the tests, so the lattice velocity is the unwrapped displacement.
 * Output n[site][Q] (overwritten). */
int orc_ni_literal(const orc_lattice *L, int dim, int n, const double *xu_prev,
                   const double *xu_now, uint64_t *nout)
{
    int W = 2 * L->V + 1;
    int Q = 1;
    long nsite = 1;
    double box[3];
    for (int a = 0; a < dim; ++a) {
        Q *= W;
        nsite *= L->M[a];
        box[a] = L->M[a] * L->dx;
    }
    memset(nout, 0, sizeof(uint64_t) * (size_t)nsite * Q);
    for (long site = 0; site < nsite; ++site) {
        long xs[3] = {0, 0, 0};
        long r = site;
        for (int a = 0; a < dim; ++a) {
            xs[a] = r % L->M[a];
            r /= L->M[a];
        }
        for (int i = 0; i < Q; ++i) {
            long vi[3] = {0, 0, 0};
            long q = i;
            for (int a = 0; a < dim; ++a) {
                vi[a] = q % W - L->V;
                q /= W;
            }
            for (int j = 0; j < n; ++j) {
                int in_now = 1, in_prev = 1;
                for (int a = 0; a < dim; ++a) {
                    double shift = box[a] * floor(xu_now[j * dim + a] / box[a]);
                    double xn = xu_now[j * dim + a] - shift;
                    double xp = xu_prev[j * dim + a] - shift;
                    double lo = xs[a] * L->dx;
                    if (!(lo <= xn && xn < lo + L->dx))
                        in_now = 0;
                    double lop = (xs[a] - vi[a]) * L->dx;
                    if (!(lop <= xp && xp < lop + L->dx))
                        in_prev = 0;
                }
                nout[site * Q + i] += (uint64_t)(in_now * in_prev);
            }
        }
    }
    return ORC_OK;
}

/* Full MDLG run: n_lattice lattice steps of md_per_lattice velocity-Verlet
 * steps each, binning after every lattice step against the snapshot of the
 * previous one (the first snapshot is the state on entry).  Accumulates into
 * A, mom, dsum, dsq.  When hist_t is not NULL it receives, per lattice step,
 * the site-summed counts n_i (n_lattice x Q) for batch-mean error bars.
 * On entry acc must hold a(t) for x(t). */
int orc_mdlg_run(const orc_md *p, const orc_lattice *L, int md_per_lattice,
                 long n_lattice, double *x, int32_t *img, double *v,
                 double *acc, long *step, int use_cells, uint64_t *A,
                 int64_t *mom, double *dsum, double *dsq, uint64_t *hist_t)
{
    int d = p->dim, n = p->n;
    int W = 2 * L->V + 1;
    int Q = 1;
    long nsite = 1;
    for (int a = 0; a < d; ++a) {
        Q *= W;
        nsite *= L->M[a];
    }
    double *prev = (double *)malloc(sizeof(double) * (size_t)n * d);
    double *now = (double *)malloc(sizeof(double) * (size_t)n * d);
    uint64_t *tmp = hist_t ? (uint64_t *)calloc((size_t)nsite * Q, sizeof(uint64_t)) : NULL;
    if (!prev || !now || (hist_t && !tmp)) {
        free(prev); free(now); free(tmp);
        return ORC_ENOMEM;
    }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a)
            prev[i * d + a] = x[i * d + a] + img[i * d + a] * p->box[a];
    int rc = ORC_OK;
    for (long t = 0; t < n_lattice; ++t) {
        rc = orc_vv(p, x, img, v, acc, md_per_lattice, step, 0, 0.0, use_cells);
        if (rc != ORC_OK)
            break;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < d; ++a)
                now[i * d + a] = x[i * d + a] + img[i * d + a] * p->box[a];
        if (hist_t) {
            int nm = orc_num_moments(d);
            int64_t *mtmp = (int64_t *)calloc((size_t)nsite * nm, sizeof(int64_t));
            double ds[3] = {0, 0, 0}, dq[3] = {0, 0, 0};
            if (!mtmp) { rc = ORC_ENOMEM; break; }
            memset(tmp, 0, sizeof(uint64_t) * (size_t)nsite * Q);
            orc_bin(L, d, n, prev, now, tmp, mtmp, ds, dq);
            for (int i = 0; i < Q; ++i) {
                uint64_t s = 0;
                for (long st = 0; st < nsite; ++st)
                    s += tmp[st * Q + i];
                hist_t[t * Q + i] = s;
            }
            free(mtmp);
        }
        orc_bin(L, d, n, prev, now, A, mom, dsum, dsq);
        double *sw = prev;
        prev = now;
        now = sw;
    }
    free(prev);
    free(now);
    free(tmp);
    return rc;
}

/* Thermostatted equilibration as the configurations prescribe: nsteps
 * velocity-Verlet steps, rescaling to kT every thermo_every steps. */
int orc_equilibrate(const orc_md *p, double *x, int32_t *img, double *v,
                    double *acc, long nsteps, long *step, int thermo_every,
                    double kT, int use_cells)
{
    return orc_vv(p, x, img, v, acc, nsteps, step, thermo_every, kT, use_cells);
}

/* Kinetic energy sum (1/2) m v^2 and total momentum sum m v (FP64). */
void orc_kinetics(const orc_md *p, const double *v, double *ke, double *mom)
{
    int d = p->dim;
    *ke = 0.0;
    for (int a = 0; a < d; ++a)
        mom[a] = 0.0;
    for (int i = 0; i < p->n; ++i)
        for (int a = 0; a < d; ++a) {
            *ke += 0.5 * p->mass * v[i * d + a] * v[i * d + a];
            mom[a] += p->mass * v[i * d + a];
        }
}

/* ------------------------------------------------------------------ */
/* Adjoint of a velocity-Verlet window (gradients of displacement     */
/* moments with respect to eps, sigma and the initial velocities)     */
/* ------------------------------------------------------------------ */

/* For every ordered pair (i, j) within r_c, with r = x_i - x_j (minimum image):
 *   acceleration      a_i      += g(r) r / m,
 *                     g(r)      = (24 eps / r^2) [2 (sigma/r)^12 - (sigma/r)^6]
 *   sigma derivative  da_i/dsig += (dg/dsigma) r / m,
 *                     dg/dsigma = (24 eps / (r^2 sigma)) [24 (sigma/r)^12 - 6 (sigma/r)^6]
 *   Jacobian-vector   (J lam)_i += K (lam_i - lam_j) / m,
 *                     K = g I + (g'(r)/r) r r^T,
 *                     g'(r)/r   = (24 eps / r^4) [8 (sigma/r)^6 - 28 (sigma/r)^12].
 * Any of the outputs may be NULL. */
typedef struct {
    const orc_md *p;
    const double *lam;
    double *acc, *dacc, *jlam;
} pair_terms_ctx;

static void pair_terms_fn(void *vctx, int i, int j, const double *r, double r2)
{
    pair_terms_ctx *c = (pair_terms_ctx *)vctx;
    const orc_md *p = c->p;
    int d = p->dim;
    double eps = p->eps, sig = p->sigma, m = p->mass;
    double rr = sqrt(r2);
    double s6 = pow(sig / rr, 6.0), s12 = s6 * s6;
    double g = 24.0 * eps / r2 * (2.0 * s12 - s6);
    if (c->acc)
        for (int a = 0; a < d; ++a)
            c->acc[i * d + a] += g * r[a] / m;
    if (c->dacc) {
        double dg = 24.0 * eps / (r2 * sig) * (24.0 * s12 - 6.0 * s6);
        for (int a = 0; a < d; ++a)
            c->dacc[i * d + a] += dg * r[a] / m;
    }
    if (c->jlam) {
        double gp = 24.0 * eps / (r2 * r2) * (8.0 * s6 - 28.0 * s12);
        double dl[3] = {0.0, 0.0, 0.0}, rdl = 0.0;
        for (int a = 0; a < d; ++a) {
            dl[a] = c->lam[i * d + a] - c->lam[j * d + a];
            rdl += r[a] * dl[a];
        }
        for (int a = 0; a < d; ++a)
            c->jlam[i * d + a] += (g * dl[a] + gp * rdl * r[a]) / m;
    }
}

int orc_pair_terms(const orc_md *p, const double *x, const double *lam, double *acc,
                   double *dacc_dsigma, double *jlam)
{
    size_t nd = (size_t)p->n * p->dim;
    if (acc) memset(acc, 0, sizeof(double) * nd);
    if (dacc_dsigma) memset(dacc_dsigma, 0, sizeof(double) * nd);
    if (jlam) memset(jlam, 0, sizeof(double) * nd);
    if (p->forces_off)
        return ORC_OK;
    pair_terms_ctx c = {p, lam, acc, dacc_dsigma, jlam};
    return visit_pairs(p, x, pair_terms_fn, &c);
}

/* Loss on the displacement over the window (unwrapped positions):
 *   loss_id 0: L = (1/(N d)) sum_j |x_j(W) - x_j(0)|^2   (per-axis MSD)
 *   loss_id 1: L = (1/N) sum_j (x_jx(W) - x_jx(0))       (mean x displacement)
 * Writes L and dL/dx(W) into lx. */
static double window_loss(int loss_id, int n, int d, const double *xu0, const double *xuW,
                          double *lx)
{
    double L = 0.0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a) {
            double dd = xuW[i * d + a] - xu0[i * d + a];
            if (loss_id == 0) {
                L += dd * dd / ((double)n * d);
                if (lx) lx[i * d + a] = 2.0 * dd / ((double)n * d);
            } else {
                if (a == 0) L += dd / n;
                if (lx) lx[i * d + a] = (a == 0) ? 1.0 / n : 0.0;
            }
        }
    return L;
}

/* Forward window of W velocity-Verlet steps from (x0 wrapped in [0, L), v0),
 * then the reverse sweep.  With the step written as kick (h/2) a(x_n),
 * drift h v, kick (h/2) a(x_{n+1}), the adjoints (lx, lv) of (x, v) run
 * backwards as: lv += h lx (drift); at every position the two half kicks that
 * use a(x_n) add c J(x_n)^T lv to lx and c lv . da(x_n)/dtheta to the
 * parameter gradients, with c = h inside the window and h/2 at both ends
 * (J is symmetric).  Outputs: *L, dL/deps, dL/dsigma, dL/dv0 [n][d] and,
 * when gx0 is not NULL, dL/dx0. */
int orc_adjoint(const orc_md *p, const double *x0, const double *v0, int W, int loss_id,
                double *L, double *geps, double *gsig, double *gv0, double *gx0)
{
    int d = p->dim, n = p->n;
    size_t nd = (size_t)n * d;
    double h = p->dt;
    double *xs = (double *)malloc(sizeof(double) * nd * (size_t)(W + 1)); /* wrapped */
    double *xu = (double *)malloc(sizeof(double) * nd * 2);               /* unwrapped x0, xW */
    double *x = (double *)malloc(sizeof(double) * nd);
    double *v = (double *)malloc(sizeof(double) * nd);
    double *acc = (double *)malloc(sizeof(double) * nd);
    double *lx = (double *)malloc(sizeof(double) * nd);
    double *lv = (double *)calloc(nd, sizeof(double));
    double *t1 = (double *)malloc(sizeof(double) * nd);
    double *t2 = (double *)malloc(sizeof(double) * nd);
    int32_t *img = (int32_t *)calloc(nd, sizeof(int32_t));
    if (!xs || !xu || !x || !v || !acc || !lx || !lv || !t1 || !t2 || !img) {
        free(xs); free(xu); free(x); free(v); free(acc); free(lx); free(lv); free(t1);
        free(t2); free(img);
        return ORC_ENOMEM;
    }
    memcpy(x, x0, sizeof(double) * nd);
    memcpy(v, v0, sizeof(double) * nd);
    memcpy(xs, x0, sizeof(double) * nd);
    memcpy(xu, x0, sizeof(double) * nd);
    orc_pair_terms(p, x, NULL, acc, NULL, NULL);
    long step = 0;
    for (int s = 1; s <= W; ++s) {
        orc_vv(p, x, img, v, acc, 1, &step, 0, 0.0, 1);
        memcpy(xs + nd * (size_t)s, x, sizeof(double) * nd);
    }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a)
            xu[nd + i * d + a] = x[i * d + a] + img[i * d + a] * p->box[a];
    double Lv = window_loss(loss_id, n, d, xu, xu + nd, lx);
    double ge = 0.0, gs = 0.0;
    for (int s = W; s >= 0; --s) {
        double c = (s == W || s == 0) ? 0.5 * h : h;
        const double *xn = xs + nd * (size_t)s;
        orc_pair_terms(p, xn, lv, acc, t1, t2);
        for (size_t k = 0; k < nd; ++k) {
            lx[k] += c * t2[k];
            ge += c * lv[k] * acc[k] / p->eps;
            gs += c * lv[k] * t1[k];
        }
        if (s > 0)
            for (size_t k = 0; k < nd; ++k)
                lv[k] += h * lx[k];
    }
    if (L) *L = Lv;
    if (geps) *geps = ge;
    if (gsig) *gsig = gs;
    if (gv0) memcpy(gv0, lv, sizeof(double) * nd);
    if (gx0) memcpy(gx0, lx, sizeof(double) * nd);
    free(xs); free(xu); free(x); free(v); free(acc); free(lx); free(lv); free(t1); free(t2);
    free(img);
    return ORC_OK;
}

/* The window loss alone (forward only), for finite differences. */
int orc_window_loss(const orc_md *p, const double *x0, const double *v0, int W, int loss_id,
                    double *L)
{
    int d = p->dim, n = p->n;
    size_t nd = (size_t)n * d;
    double *x = (double *)malloc(sizeof(double) * nd);
    double *v = (double *)malloc(sizeof(double) * nd);
    double *acc = (double *)malloc(sizeof(double) * nd);
    double *xuW = (double *)malloc(sizeof(double) * nd);
    int32_t *img = (int32_t *)calloc(nd, sizeof(int32_t));
    if (!x || !v || !acc || !xuW || !img) {
        free(x); free(v); free(acc); free(xuW); free(img);
        return ORC_ENOMEM;
    }
    memcpy(x, x0, sizeof(double) * nd);
    memcpy(v, v0, sizeof(double) * nd);
    orc_pair_terms(p, x, NULL, acc, NULL, NULL);
    long step = 0;
    orc_vv(p, x, img, v, acc, W, &step, 0, 0.0, 1);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a)
            xuW[i * d + a] = x[i * d + a] + img[i * d + a] * p->box[a];
    *L = window_loss(loss_id, n, d, x0, xuW, NULL);
    free(x); free(v); free(acc); free(xuW); free(img);
    return ORC_OK;
}
