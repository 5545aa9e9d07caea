/*
 * pic_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Slow on purpose: every loop is written the way the method is stated, with
 * no blocking, fusion or reordering.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never
 * does.  It shares no code with the GPU library.
 *
 * Paper sections followed: Section 2 (gather/deposit stencils and staggering),
 * Section 3 (boundaries, secondary emission, collision processes and
 * thresholds, neutral background), Section 4 (seed load, external circuit).
 * The paper does not print its field solver, circuit law, collision kinematics
 * or random-number scheme; the readings used here are restated at each
 * function.
 *
 * Parity status: every function below is pinned by a CPU test against a
 * closed form, an invariant, a library routine or brute force.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 */
static const double EPS0 = 8.8541878128e-12;
static const double QE = 1.602176634e-19;
static const double KB = 1.380649e-23;
static const double PI = 3.14159265358979323846;

#define IDX(p, i, j) ((int64_t)(j) * ((p)->nr + 1) + (i))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the round function published by Salmon et al. (SC'11): */
/* each round multiplies words 0 and 2 by the two round multipliers, and      */
/* mixes the high halves with words 1, 3 and the key; the key is bumped by the */
/* Weyl constants between rounds.                                              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Random stream layout: counter = (particle id, run<<8 | species<<4 | purpose,
 * step, 0); key = the 64-bit seed split low/high. */
enum { PUR_MCC = 0, PUR_IZ = 1, PUR_ION = 2, PUR_SEE = 3 };

static void draw(const orc_problem *p, uint32_t id, int species, int purpose,
                 int64_t step, uint32_t u[4])
{
    uint32_t c[4], k[2];
    c[0] = id;
    c[1] = (p->run << 8) | ((uint32_t)species << 4) | (uint32_t)purpose;
    c[2] = (uint32_t)step;
    c[3] = 0;
    k[0] = (uint32_t)(p->seed & 0xffffffffu);
    k[1] = (uint32_t)(p->seed >> 32);
    orc_philox4x32_10(c, k, u);
}

/* Uniform on [0,1) from the top 24 bits (exact in binary32 and binary64). */
static double u24(uint32_t u) { return (double)(u >> 8) * (1.0 / 16777216.0); }
/* Uniform on (0,1) for log(): midpoint of a 23-bit cell, so that the value
 * is exact in binary32 as well as binary64. */
static double u_open(uint32_t u) { return ((double)(u >> 9) + 0.5) * (1.0 / 8388608.0); }

/* ------------------------------------------------------------------------ */
/* Field solve.                                                              */
/*                                                                           */
/* Reading of "Gauss' law is obeyed along this axis" (Section 3): charge-form */
/* finite volumes.  Node (i,j) owns [r_{i-1/2}, r_{i+1/2}] x [z_{j-1/2},      */
/* z_{j+1/2}] clipped to the domain (r_{-1/2} = 0).  Across each face f the   */
/* flux is eps0 * A_f * (phi_node - phi_nb) / h_f and the fluxes out of a     */
/* control volume sum to the node charge Q_ij (Gauss).  The axis has no face, */
/* so its Neumann condition is built in.                                      */
/* ------------------------------------------------------------------------ */

int orc_node_kind(const orc_problem *p, int i, int j)
{
    double r = i * (p->lr / p->nr);
    if (j == p->nz || i == p->nr) return 2;              /* anode, outer wall */
    if (j == 0 && r < p->cathode_rmax) return 1;          /* cathode           */
    return 0;                                             /* unknown (incl. the Neumann block at z = 0) */
}

/* c_east[n]: coupling eps0*A/h across the face between (i,j) and (i+1,j);
 * c_north[n]: between (i,j) and (i,j+1).  Zero where the face does not exist. */
void orc_couplings(const orc_problem *p, double *c_east, double *c_north)
{
    const double dr = p->lr / p->nr, dz = p->lz / p->nz;
    for (int j = 0; j <= p->nz; ++j) {
        for (int i = 0; i <= p->nr; ++i) {
            int64_t n = IDX(p, i, j);
            /* radial face at r_{i+1/2}, spanning the node's clipped z-extent */
            if (i < p->nr) {
                double dzj = (j == 0 || j == p->nz) ? 0.5 * dz : dz;
                double rf = (i + 0.5) * dr;
                double area = 2.0 * PI * rf * dzj;
                c_east[n] = EPS0 * area / dr;
            } else {
                c_east[n] = 0.0;
            }
            /* axial face at z_{j+1/2}: the annulus of the node's r-extent */
            if (j < p->nz) {
                double rlo = (i == 0) ? 0.0 : (i - 0.5) * dr;
                double rhi = (i == p->nr) ? p->lr : (i + 0.5) * dr;
                double area = PI * (rhi * rhi - rlo * rlo);
                c_north[n] = EPS0 * area / dz;
            } else {
                c_north[n] = 0.0;
            }
        }
    }
}

/* (K phi)_n = sum over the node's faces of c_f (phi_n - phi_nb), every node. */
void orc_apply_k_full(const orc_problem *p, const double *phi, double *out)
{
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    double *ce = malloc(sizeof(double) * nn), *cn = malloc(sizeof(double) * nn);
    orc_couplings(p, ce, cn);
    for (int j = 0; j <= p->nz; ++j) {
        for (int i = 0; i <= p->nr; ++i) {
            int64_t n = IDX(p, i, j);
            double s = 0.0;
            if (i < p->nr) s += ce[n] * (phi[n] - phi[IDX(p, i + 1, j)]);
            if (i > 0) s += ce[IDX(p, i - 1, j)] * (phi[n] - phi[IDX(p, i - 1, j)]);
            if (j < p->nz) s += cn[n] * (phi[n] - phi[IDX(p, i, j + 1)]);
            if (j > 0) s += cn[IDX(p, i, j - 1)] * (phi[n] - phi[IDX(p, i, j - 1)]);
            out[n] = s;
        }
    }
    free(ce);
    free(cn);
}

/* Field energy W = 1/2 sum over faces of c_f (delta phi)^2 = 1/2 phi^T K phi. */
double orc_field_energy(const orc_problem *p, const double *phi)
{
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    double *ce = malloc(sizeof(double) * nn), *cn = malloc(sizeof(double) * nn);
    orc_couplings(p, ce, cn);
    double w = 0.0;
    for (int j = 0; j <= p->nz; ++j)
        for (int i = 0; i <= p->nr; ++i) {
            int64_t n = IDX(p, i, j);
            if (i < p->nr) { double d = phi[n] - phi[IDX(p, i + 1, j)]; w += 0.5 * ce[n] * d * d; }
            if (j < p->nz) { double d = phi[n] - phi[IDX(p, i, j + 1)]; w += 0.5 * cn[n] * d * d; }
        }
    free(ce);
    free(cn);
    return w;
}

static int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_thread_count(void)
{
    return orc_threads();
}

static int orc_thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* Sums taken over [0, nn) in the solver: each thread sums one contiguous
 * range in order, and the per-thread partial sums are added in thread
 * order.  Deterministic for a given thread count; with one thread it is the
 * plain loop. */
#define THREAD_RANGE(nn, lo, hi)                                              \
    const int nthr_ = omp_team_size();                                        \
    const int t_ = orc_thread_id();                                           \
    const int64_t lo = (nn) * t_ / nthr_, hi = (nn) * (t_ + 1) / nthr_

static int omp_team_size(void)
{
#ifdef _OPENMP
    return omp_get_num_threads();
#else
    return 1;
#endif
}

static double sum_parts(const double *part, int nthr, int stride, int k)
{
    double s = 0.0;
    for (int t = 0; t < nthr; ++t) s += part[t * stride + k];
    return s;
}

/* Solve for phi with cathode nodes at v_cathode, grounded nodes at 0 and the
 * unknown rows satisfying (K phi)_u = Q_u.  Jacobi-preconditioned conjugate
 * gradients on the unknowns, warm-started from phi, until
 * ||b - K_uu phi_u|| <= rtol ||b||.  Returns 0 on convergence, -4 otherwise. */
int orc_solve(const orc_problem *p, const double *q_node, double v_cathode,
              double *phi, double rtol, int maxit, int64_t *iters, double *rel_res)
{
    const int nr = p->nr, nz = p->nz;
    int64_t nn = (int64_t)(nr + 1) * (nz + 1);
    double *ce = malloc(sizeof(double) * nn), *cn = malloc(sizeof(double) * nn);
    double *b = calloc(nn, sizeof(double)), *r = calloc(nn, sizeof(double));
    double *z = calloc(nn, sizeof(double)), *d = calloc(nn, sizeof(double));
    double *q = calloc(nn, sizeof(double)), *dg = calloc(nn, sizeof(double));
    char *kind = malloc(nn);
    orc_couplings(p, ce, cn);
    for (int j = 0; j <= nz; ++j)
        for (int i = 0; i <= nr; ++i) {
            int64_t n = IDX(p, i, j);
            kind[n] = (char)orc_node_kind(p, i, j);
            if (kind[n] == 1) phi[n] = v_cathode;
            if (kind[n] == 2) phi[n] = 0.0;
        }
    /* Right-hand side: node charge plus couplings to Dirichlet neighbours;
     * diagonal: sum of all couplings of the node. */
    for (int j = 0; j <= nz; ++j)
        for (int i = 0; i <= nr; ++i) {
            int64_t n = IDX(p, i, j);
            if (kind[n] != 0) continue;
            double s = q_node[n], diag = 0.0;
            int64_t nb[4]; double c[4]; int k = 0;
            if (i < nr) { nb[k] = IDX(p, i + 1, j); c[k++] = ce[n]; }
            if (i > 0) { nb[k] = IDX(p, i - 1, j); c[k++] = ce[IDX(p, i - 1, j)]; }
            if (j < nz) { nb[k] = IDX(p, i, j + 1); c[k++] = cn[n]; }
            if (j > 0) { nb[k] = IDX(p, i, j - 1); c[k++] = cn[IDX(p, i, j - 1)]; }
            for (int t = 0; t < k; ++t) {
                diag += c[t];
                if (kind[nb[t]] != 0) s += c[t] * phi[nb[t]];
            }
            b[n] = s;
            dg[n] = diag;
        }
    /* Operator rows of the unknowns in flux form, y_m = sum_f c_f (x_m - x_nb).
     * Applied to phi (Dirichlet values in place) it gives K phi on the
     * unknown rows; applied to a vector that is zero on Dirichlet nodes it is
     * the matrix K_uu.  The differences are formed before scaling, which keeps
     * round-off small for smooth potentials. */
#define APPLY(x, y)                                                          \
    _Pragma("omp parallel for schedule(static)")                              \
    for (int jj = 0; jj <= nz; ++jj)                                          \
        for (int ii = 0; ii <= nr; ++ii) {                                    \
            int64_t m = IDX(p, ii, jj);                                       \
            if (kind[m] != 0) { y[m] = 0.0; continue; }                       \
            double acc = 0.0;                                                 \
            if (ii < nr) acc += ce[m] * (x[m] - x[IDX(p, ii + 1, jj)]);        \
            if (ii > 0) acc += ce[IDX(p, ii - 1, jj)] * (x[m] - x[IDX(p, ii - 1, jj)]); \
            if (jj < nz) acc += cn[m] * (x[m] - x[IDX(p, ii, jj + 1)]);        \
            if (jj > 0) acc += cn[IDX(p, ii, jj - 1)] * (x[m] - x[IDX(p, ii, jj - 1)]); \
            y[m] = acc;                                                       \
        }

    const int nthr = orc_threads();
    double *part = calloc((size_t)nthr * 2, sizeof(double));
#pragma omp parallel num_threads(nthr)
    {
        THREAD_RANGE(nn, lo, hi);
        double s = 0.0;
        for (int64_t n = lo; n < hi; ++n) s += b[n] * b[n];
        part[2 * t_] = s;
    }
    double bnorm = sqrt(sum_parts(part, nthr, 2, 0));
    int status = 0;
    int64_t it = 0;
    double res = 0.0;
    if (bnorm == 0.0) {
        for (int64_t n = 0; n < nn; ++n) if (kind[n] == 0) phi[n] = 0.0;
    } else {
        /* CG restarted from the true residual b - A phi until that residual
         * itself meets the tolerance (the recursively updated residual can
         * drift from it at very tight tolerances). */
        double last = HUGE_VAL;
        for (int restart = 0;; ++restart) {
            APPLY(phi, q);
#pragma omp parallel num_threads(nthr)
            {
                THREAD_RANGE(nn, lo, hi);
                double s_rz = 0.0, s_rr = 0.0;
                for (int64_t n = lo; n < hi; ++n) {
                    r[n] = (kind[n] == 0) ? q_node[n] - q[n] : 0.0;
                    z[n] = (kind[n] == 0) ? r[n] / dg[n] : 0.0;
                    d[n] = z[n];
                    s_rz += r[n] * z[n];
                    s_rr += r[n] * r[n];
                }
                part[2 * t_] = s_rz;
                part[2 * t_ + 1] = s_rr;
            }
            double rz = sum_parts(part, nthr, 2, 0), rr = sum_parts(part, nthr, 2, 1);
            res = sqrt(rr) / bnorm;
            /* stop when converged, out of iterations, or when a restart no
             * longer reduces the true residual (round-off floor) */
            if (res <= rtol || it >= maxit || (restart > 0 && res >= 0.5 * last)) break;
            last = res;
            double rec = res;
            while (rec > 0.5 * rtol && it < maxit) {
                APPLY(d, q);
#pragma omp parallel num_threads(nthr)
                {
                    THREAD_RANGE(nn, lo, hi);
                    double s = 0.0;
                    for (int64_t n = lo; n < hi; ++n) s += d[n] * q[n];
                    part[2 * t_] = s;
                }
                double alpha = rz / sum_parts(part, nthr, 2, 0);
#pragma omp parallel num_threads(nthr)
                {
                    THREAD_RANGE(nn, lo, hi);
                    double s_rz = 0.0, s_rr = 0.0;
                    for (int64_t n = lo; n < hi; ++n) {
                        if (kind[n] != 0) continue;
                        phi[n] += alpha * d[n];
                        r[n] -= alpha * q[n];
                        z[n] = r[n] / dg[n];
                        s_rz += r[n] * z[n];
                        s_rr += r[n] * r[n];
                    }
                    part[2 * t_] = s_rz;
                    part[2 * t_ + 1] = s_rr;
                }
                double rz_new = sum_parts(part, nthr, 2, 0);
                rr = sum_parts(part, nthr, 2, 1);
                double beta = rz_new / rz;
                rz = rz_new;
#pragma omp parallel for schedule(static) num_threads(nthr)
                for (int64_t n = 0; n < nn; ++n) d[n] = z[n] + beta * d[n];
                ++it;
                rec = sqrt(rr) / bnorm;
            }
        }
        if (res > rtol) status = -4;
    }
#undef APPLY
    if (iters) *iters = it;
    if (rel_res) *rel_res = res;
    free(ce); free(cn); free(b); free(r); free(z); free(d); free(q); free(dg); free(kind);
    free(part);
    return status;
}

/* MC-PIC nodal field: centred differences of -grad(phi) inside, E_r = 0 on the
 * axis, one-sided differences on the walls. */
void orc_nodal_e(const orc_problem *p, const double *phi, double *er, double *ez)
{
    const double dr = p->lr / p->nr, dz = p->lz / p->nz;
    for (int j = 0; j <= p->nz; ++j)
        for (int i = 0; i <= p->nr; ++i) {
            int64_t n = IDX(p, i, j);
            if (i == 0) er[n] = 0.0;
            else if (i == p->nr) er[n] = -(phi[n] - phi[IDX(p, i - 1, j)]) / dr;
            else er[n] = -(phi[IDX(p, i + 1, j)] - phi[IDX(p, i - 1, j)]) / (2.0 * dr);
            if (j == 0) ez[n] = -(phi[IDX(p, i, 1)] - phi[n]) / dz;
            else if (j == p->nz) ez[n] = -(phi[n] - phi[IDX(p, i, j - 1)]) / dz;
            else ez[n] = -(phi[IDX(p, i, j + 1)] - phi[IDX(p, i, j - 1)]) / (2.0 * dz);
        }
}

/* Node volumes: a tent weight S_i(r) S_j(z) integrated over the cylinder.
 * In r, the integral of 2 pi r S_i(r) dr is pi dr^2 / 3 on the axis,
 * 2 pi r_i dr inside and pi dr R - pi dr^2 / 3 at the outer wall; in z it is
 * dz inside and dz / 2 on the two z walls. */
void orc_node_volumes(const orc_problem *p, double *vol)
{
    const double dr = p->lr / p->nr, dz = p->lz / p->nz;
    for (int j = 0; j <= p->nz; ++j)
        for (int i = 0; i <= p->nr; ++i) {
            double a;
            if (i == 0) a = PI * dr * dr / 3.0;
            else if (i == p->nr) a = PI * dr * p->lr - PI * dr * dr / 3.0;
            else a = 2.0 * PI * (i * dr) * dr;
            double h = (j == 0 || j == p->nz) ? 0.5 * dz : dz;
            vol[IDX(p, i, j)] = a * h;
        }
}

/* Cell and in-cell fraction of a position: i = floor(r/dr) kept in
 * [0, nr-1], f = r/dr - i (likewise in z). */
static void locate(const orc_problem *p, double r, double z, int *i, int *j, double *fr, double *fz)
{
    double x = r / (p->lr / p->nr), y = z / (p->lz / p->nz);
    int ii = (int)floor(x), jj = (int)floor(y);
    if (ii < 0) ii = 0;
    if (ii > p->nr - 1) ii = p->nr - 1;
    if (jj < 0) jj = 0;
    if (jj > p->nz - 1) jj = p->nz - 1;
    *i = ii; *j = jj; *fr = x - ii; *fz = y - jj;
}

/* Linear (tent) deposit, Section 2: node (i,j) receives q w S_i(r) S_j(z). */
void orc_deposit(const orc_problem *p, const double *r, const double *z, int64_t n,
                 double qw, double *q_node)
{
    for (int64_t k = 0; k < n; ++k) {
        int i, j; double fr, fz;
        locate(p, r[k], z[k], &i, &j, &fr, &fz);
        q_node[IDX(p, i, j)] += qw * (1.0 - fr) * (1.0 - fz);
        q_node[IDX(p, i + 1, j)] += qw * fr * (1.0 - fz);
        q_node[IDX(p, i, j + 1)] += qw * (1.0 - fr) * fz;
        q_node[IDX(p, i + 1, j + 1)] += qw * fr * fz;
    }
}

/* Field at a particle (Section 2).
 * EC-PIC: E_r lives on r-edges and is taken NGP in r (the edge of the
 *   particle's cell), linear in z; E_z lives on z-edges, linear in r, NGP in z.
 *   Written out, this is minus the gradient of the bilinear interpolant of phi.
 * MC-PIC: the nodal field above, interpolated with the deposit's tent weights.
 * B: tent-weighted nodal B in both schemes. */
static void field_at(const orc_problem *p, const double *phi, const double *ern,
                     const double *ezn, double r, double z,
                     double *er, double *ez, double *br, double *bz)
{
    const double dr = p->lr / p->nr, dz = p->lz / p->nz;
    int i, j; double fr, fz;
    locate(p, r, z, &i, &j, &fr, &fz);
    int64_t n00 = IDX(p, i, j), n10 = IDX(p, i + 1, j);
    int64_t n01 = IDX(p, i, j + 1), n11 = IDX(p, i + 1, j + 1);
    double w00 = (1 - fr) * (1 - fz), w10 = fr * (1 - fz), w01 = (1 - fr) * fz, w11 = fr * fz;
    if (p->scheme == 1) {
        double er_lo = -(phi[n10] - phi[n00]) / dr;   /* edge ((i+1/2), j)   */
        double er_hi = -(phi[n11] - phi[n01]) / dr;   /* edge ((i+1/2), j+1) */
        double ez_lo = -(phi[n01] - phi[n00]) / dz;   /* edge (i, j+1/2)     */
        double ez_hi = -(phi[n11] - phi[n10]) / dz;   /* edge (i+1, j+1/2)   */
        *er = (1 - fz) * er_lo + fz * er_hi;
        *ez = (1 - fr) * ez_lo + fr * ez_hi;
    } else {
        *er = w00 * ern[n00] + w10 * ern[n10] + w01 * ern[n01] + w11 * ern[n11];
        *ez = w00 * ezn[n00] + w10 * ezn[n10] + w01 * ezn[n01] + w11 * ezn[n11];
    }
    *br = w00 * p->b_r[n00] + w10 * p->b_r[n10] + w01 * p->b_r[n01] + w11 * p->b_r[n11];
    *bz = w00 * p->b_z[n00] + w10 * p->b_z[n10] + w01 * p->b_z[n01] + w11 * p->b_z[n11];
}

void orc_gather(const orc_problem *p, const double *phi, const double *r, const double *z,
                int64_t n, double *er, double *ez, double *br, double *bz)
{
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    double *ern = malloc(sizeof(double) * nn), *ezn = malloc(sizeof(double) * nn);
    orc_nodal_e(p, phi, ern, ezn);
    for (int64_t k = 0; k < n; ++k)
        field_at(p, phi, ern, ezn, r[k], z[k], &er[k], &ez[k], &br[k], &bz[k]);
    free(ern);
    free(ezn);
}

/* ------------------------------------------------------------------------ */
/* Null-collision Monte Carlo (Section 3, processes (1a)-(1d)).              */
/* nu_j(E) = n_g sigma_j(E) sqrt(2 e E / m_e) on the table's energies;       */
/* nu_max = max over table energies of the summed frequency (an upper bound   */
/* of the piecewise-linear interpolant); P_null = 1 - exp(-nu_max dt).        */
/* ------------------------------------------------------------------------ */
double orc_nu_tables(const orc_problem *p, double *nu, uint64_t *t_null)
{
    double ng = p->p_gas / (KB * p->t_gas);
    double numax = 0.0;
    for (int k = 0; k < p->n_table; ++k) {
        double e = k * p->de_table;
        double v = sqrt(2.0 * QE * e / p->m[0]);
        double sum = 0.0;
        for (int c = 0; c < 4; ++c) {
            /* processes (1a)-(1c) collide with ground-state argon, (1d) with
             * the static metastable density */
            double target = (c < 3) ? ng : p->n_meta;
            nu[c * p->n_table + k] = target * p->sigma[c * p->n_table + k] * v;
            sum += nu[c * p->n_table + k];
        }
        if (sum > numax) numax = sum;
    }
    double pnull = 1.0 - exp(-numax * p->dt);
    if (t_null) *t_null = (uint64_t)floor(pnull * 4294967296.0);
    return numax;
}

/* Linear interpolation of a table row at E (eV); clamped above the top. */
static double interp(const double *row, int n, double de, double e)
{
    double x = e / de;
    int k;
    double f;
    if (x >= (double)(n - 1)) { k = n - 2; f = 1.0; }
    else { k = (int)floor(x); f = x - k; }
    return (1.0 - f) * row[k] + f * row[k + 1];
}

/* Null-collision selection (one electron, after its push): it is a
 * candidate iff the first word of its collision draw is below
 * floor(P_null 2^32) (an integer test); a candidate's process follows from
 * R = U24(u1) nu_max against the cumulative frequencies nu_el, + nu_ex,
 * + nu_iz at its energy; a selected inelastic process below its threshold,
 * and anything beyond the sum, is a null collision. */
int orc_mcc_select(const orc_problem *p, const double *nu, double numax, uint64_t t_null,
                   uint32_t id, int64_t step, double vr, double vt, double vz, double *margin)
{
    uint32_t u[4];
    draw(p, id, 0, PUR_MCC, step, u);
    if (margin) *margin = 0.0;
    if ((uint64_t)u[0] >= t_null) return -2;
    const double *nel = nu, *nex = nu + p->n_table, *niz = nu + 2 * p->n_table;
    const double *nmi = nu + 3 * p->n_table;
    double e = 0.5 * p->m[0] * (vr * vr + vt * vt + vz * vz) / QE;
    double c1 = interp(nel, p->n_table, p->de_table, e);
    double c2 = c1 + interp(nex, p->n_table, p->de_table, e);
    double c3 = c2 + interp(niz, p->n_table, p->de_table, e);
    double c4 = c3 + interp(nmi, p->n_table, p->de_table, e);
    double rsel = u24(u[1]) * numax;
    int proc = -1;
    if (rsel < c1) proc = 0;
    else if (rsel < c2) proc = (e >= p->e_exc) ? 1 : -1;
    else if (rsel < c3) proc = (e >= p->e_iz) ? 2 : -1;
    else if (rsel < c4) proc = (e >= p->e_iz_meta) ? 3 : -1;
    if (margin) {
        double m = fabs(rsel - c1) / numax;
        m = fmin(m, fabs(rsel - c2) / numax);
        m = fmin(m, fabs(rsel - c3) / numax);
        m = fmin(m, fabs(e - p->e_exc) / p->e_exc);
        m = fmin(m, fabs(e - p->e_iz) / p->e_iz);
        if (p->n_meta > 0.0) {
            m = fmin(m, fabs(rsel - c4) / numax);
            m = fmin(m, fabs(e - p->e_iz_meta) / p->e_iz_meta);
        }
        *margin = m;
    }
    return proc;
}

void orc_mcc_select_many(const orc_problem *p, int64_t step, int64_t n, const uint32_t *id,
                         const double *vr, const double *vt, const double *vz, int32_t *codes,
                         double *margins)
{
    double *nu = malloc(sizeof(double) * 4 * p->n_table);
    uint64_t t_null = 0;
    double numax = orc_nu_tables(p, nu, &t_null);
    for (int64_t k = 0; k < n; ++k)
        codes[k] = orc_mcc_select(p, nu, numax, t_null, id[k], step, vr[k], vt[k], vz[k],
                                  margins ? &margins[k] : NULL);
    free(nu);
}

/* Isotropic unit vector from two uniforms: cos(chi) = 1 - 2U, azimuth 2 pi U'. */
static void iso_dir(uint32_t ua, uint32_t ub, double d[3])
{
    double c = 1.0 - 2.0 * u24(ua);
    /* sin(chi) from (1 - c)(1 + c): both factors are exact for c = 1 - 2U */
    double s = sqrt(fmax(0.0, (1.0 - c) * (1.0 + c)));
    double ph = 2.0 * PI * u24(ub);
    d[0] = s * cos(ph);
    d[1] = s * sin(ph);
    d[2] = c;
}

/* ------------------------------------------------------------------------ */
/* Timestep                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct child {
    uint64_t key;              /* (parent species, parent id, kind) */
    int species;
    double r, z, vr, vt, vz;
} child;

typedef struct child_list { child *a; int64_t n, cap; } child_list;

static void push_child(child_list *l, child c)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 64;
        l->a = realloc(l->a, sizeof(child) * l->cap);
    }
    l->a[l->n++] = c;
}

/* Built with -fopenmp (the timing build), the particle loops run on all
 * cores: each thread takes one contiguous range of particles (static
 * schedule) and keeps its own sums, counters and new particles, which are
 * combined in thread order afterwards.  For a given thread count the result
 * is therefore deterministic; with one thread it is the serial loop. */
typedef struct thread_acc {
    double ke, pz, dq;
    int64_t n_abs[5], n_see, n_see_e, n_cand, n_coll[4];
    child_list kids;
} thread_acc;



static void append_children(child_list *to, child_list *from)
{
    for (int64_t c = 0; c < from->n; ++c) push_child(to, from->a[c]);
    free(from->a);
    from->a = NULL;
    from->n = from->cap = 0;
}

static int child_cmp(const void *a, const void *b)
{
    uint64_t x = ((const child *)a)->key, y = ((const child *)b)->key;
    return (x > y) - (x < y);
}

static uint64_t child_key(int parent_species, uint32_t parent_id, int kind)
{
    return ((uint64_t)parent_species << 33) | ((uint64_t)parent_id << 1) | (uint64_t)kind;
}

/* Cathode charge bookkeeping and phi = phi0 + V_c phi_L.
 *
 * Reading of the external circuit (Sections 3-4): the cathode is a conductor
 * with charge Q_c.  phi_L (cathode at 1 V, no charge) gives its capacitance
 * C; phi0 (cathode at 0 V, with the plasma charge) gives the induced charge
 * Q_c0 = sum over cathode nodes of (K phi0 - Q).  Charge conservation with a
 * backward-Euler resistor current (V_ext - V_c)/R:
 *     Q_c0 + C V^{n+1} = Q_c^n + dQ_conv + dt (V_ext - V^{n+1}) / R.      */
double orc_induced_charge(const orc_problem *p, const double *phi0, const double *q_node)
{
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    double *kp = malloc(sizeof(double) * nn);
    orc_apply_k_full(p, phi0, kp);
    double s = 0.0;
    for (int i = 0; i <= p->nr; ++i)
        if (orc_node_kind(p, i, 0) == 1) s += kp[IDX(p, i, 0)] - q_node[IDX(p, i, 0)];
    free(kp);
    return s;
}

double orc_capacitance(const orc_problem *p, const double *phi_l)
{
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    double *kp = malloc(sizeof(double) * nn);
    orc_apply_k_full(p, phi_l, kp);
    double s = 0.0;
    for (int i = 0; i <= p->nr; ++i)
        if (orc_node_kind(p, i, 0) == 1) s += kp[IDX(p, i, 0)];
    free(kp);
    return s;
}

/* Both species' deposit.  The timing build (-fopenmp) gives each thread a
 * contiguous range of particles and its own node array, and adds the arrays
 * in thread order (deterministic for a given thread count; the serial build
 * is the plain loop). */
static void deposit_species(const orc_problem *p, const orc_species *S, double qw, double *q)
{
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    const int nthr = orc_threads();
    memset(q, 0, sizeof(double) * nn);
    if (nthr == 1) {
        orc_deposit(p, S->r, S->z, S->n, qw, q);
        return;
    }
    double *part = calloc((size_t)nthr * nn, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        const int t = orc_thread_id();
        const int64_t lo = S->n * t / nthr, hi = S->n * (t + 1) / nthr;
        orc_deposit(p, S->r + lo, S->z + lo, hi - lo, qw, part + (size_t)t * nn);
    }
    for (int t = 0; t < nthr; ++t)
        for (int64_t n = 0; n < nn; ++n) q[n] += part[(size_t)t * nn + n];
    free(part);
}

static void deposit_all(const orc_problem *p, orc_species sp[2], double *q_e, double *q_i)
{
    deposit_species(p, &sp[0], p->q[0] * p->w[0], q_e);
    deposit_species(p, &sp[1], p->q[1] * p->w[1], q_i);
}

int orc_init(const orc_problem *p, orc_species sp[2], orc_state *st,
             double *phi, double *phi0, double *phi_l, double *q_e, double *q_i)
{
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    double *qt = malloc(sizeof(double) * nn), *zero = calloc(nn, sizeof(double));
    deposit_all(p, sp, q_e, q_i);
    for (int64_t n = 0; n < nn; ++n) qt[n] = q_e[n] + q_i[n];
    int64_t it; double res;
    int rc = 0;
    memset(phi_l, 0, sizeof(double) * nn);
    if (orc_solve(p, zero, 1.0, phi_l, p->poisson_rtol, p->poisson_maxit, &it, &res)) rc = -4;
    memset(phi0, 0, sizeof(double) * nn);
    if (orc_solve(p, qt, 0.0, phi0, p->poisson_rtol, p->poisson_maxit, &it, &res)) rc = -4;
    st->step = 0;
    st->cap_c = orc_capacitance(p, phi_l);
    st->vc = (p->circuit == 1) ? p->v_ext : p->v_fixed;
    st->qc = orc_induced_charge(p, phi0, qt) + st->cap_c * st->vc;
    for (int64_t n = 0; n < nn; ++n) phi[n] = phi0[n] + st->vc * phi_l[n];
    for (int s = 0; s < 2; ++s) {
        uint32_t mx = 0;
        for (int64_t k = 0; k < sp[s].n; ++k) if (sp[s].id[k] + 1u > mx) mx = sp[s].id[k] + 1u;
        st->next_id[s] = mx;
    }
    free(qt);
    free(zero);
    return rc;
}

/* One timestep, in this order (the paper gives none; this is the usual
 * explicit PIC-MCC cycle):
 *  1. gather E (EC or MC form) and B at x^n, Boris-rotate v^{n-1/2} -> v^{n+1/2};
 *  2. drift in Cartesian (x, y, z) = (r, 0, z) and rotate (v_r, v_theta) into
 *     the new meridional plane -- the axis reflects with no special case;
 *  3. walls: z < 0 -> cathode (if r < cathode_rmax; tally q w, ion-induced
 *     emission of an electron at rest at (r, 0)) or Neumann block; r >= R ->
 *     outer wall; z >= L -> anode (priority in that order);
 *  4. null-collision MCC for surviving electrons that existed before the step;
 *  5. new particles get ids in (parent species, parent id, kind) order and are
 *     appended; absorbed ones are removed;
 *  6. deposit, field solve with the cathode at 0 V, circuit, superposition. */
int orc_step(const orc_problem *p, orc_species sp[2], orc_state *st,
             double *phi, double *phi0, const double *phi_l, double *q_e, double *q_i,
             orc_diag *d)
{
    const double dt = p->dt, R = p->lr, L = p->lz;
    int64_t nn = (int64_t)(p->nr + 1) * (p->nz + 1);
    int rc = 0;
    memset(d, 0, sizeof(*d));

    double *ern = malloc(sizeof(double) * nn), *ezn = malloc(sizeof(double) * nn);
    orc_nodal_e(p, phi, ern, ezn);
    d->w_field = orc_field_energy(p, phi);

    double *nu = malloc(sizeof(double) * 4 * p->n_table);
    uint64_t t_null = 0;
    double numax = orc_nu_tables(p, nu, &t_null);
    /* emission probability per absorbed particle of species s: yield times
     * the weight ratio (one electron of weight w_e carries gamma w_s of
     * emitted charge), capped at 1 */
    uint64_t t_see[2];
    for (int s = 0; s < 2; ++s) {
        double g = (s == 0) ? p->gamma_e : p->gamma_i;
        double see_p = g * p->w[s] / p->w[0];
        if (see_p > 1.0) see_p = 1.0;
        if (see_p < 0.0) see_p = 0.0;
        t_see[s] = (uint64_t)floor(see_p * 4294967296.0);
    }

    child_list kids = {0, 0, 0};
    double dq = p->extra_current * dt;
    char *dead[2];
    int64_t n_pre[2];

    const int nthr = orc_threads();
    thread_acc *acc = calloc(nthr, sizeof(thread_acc));
    for (int s = 0; s < 2; ++s) {
        orc_species *S = &sp[s];
        n_pre[s] = S->n;
        dead[s] = calloc(S->n > 0 ? S->n : 1, 1);
        double qm = p->q[s] / p->m[s];
        for (int t = 0; t < nthr; ++t) {
            acc[t].ke = acc[t].pz = acc[t].dq = 0.0;
        }
        acc[0].dq = dq;   /* the serial build sums in exactly the loop order */
        const int64_t ns = S->n;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t k = 0; k < ns; ++k) {
            thread_acc *a = &acc[orc_thread_id()];
            if (s == 1 && p->frozen_ions) {
                double v2 = S->vr[k] * S->vr[k] + S->vt[k] * S->vt[k] + S->vz[k] * S->vz[k];
                a->ke += 0.5 * p->m[s] * p->w[s] * v2;
                a->pz += p->m[s] * p->w[s] * S->vz[k];
                continue;
            }
            double er, ez, br, bz;
            field_at(p, phi, ern, ezn, S->r[k], S->z[k], &er, &ez, &br, &bz);
            /* Boris: half electric kick, magnetic rotation, half kick.
             * Cartesian frame at the particle: x = r-hat, y = theta-hat. */
            double vx = S->vr[k], vy = S->vt[k], vz = S->vz[k];
            double h = 0.5 * qm * dt;
            double mx = vx + h * er, my = vy, mz = vz + h * ez;
            double tx = h * br, ty = 0.0, tz = h * bz;
            double t2 = tx * tx + ty * ty + tz * tz;
            double sx = 2.0 * tx / (1.0 + t2), sy = 2.0 * ty / (1.0 + t2), sz = 2.0 * tz / (1.0 + t2);
            double px = mx + (my * tz - mz * ty);
            double py = my + (mz * tx - mx * tz);
            double pz = mz + (mx * ty - my * tx);
            double qx = mx + (py * sz - pz * sy);
            double qy = my + (pz * sx - px * sz);
            double qz = mz + (px * sy - py * sx);
            double nx = qx + h * er, ny = qy, nz = qz + h * ez;
            a->ke += 0.5 * p->m[s] * p->w[s] * (vx * nx + vy * ny + vz * nz);
            a->pz += p->m[s] * p->w[s] * nz;
            /* drift and rotation into the new meridional plane */
            double x1 = S->r[k] + nx * dt, y1 = ny * dt, z1 = S->z[k] + nz * dt;
            double r1 = sqrt(x1 * x1 + y1 * y1);
            double vr1 = nx, vt1 = ny;
            if (r1 > 0.0) {
                double c = x1 / r1, sn = y1 / r1;
                vr1 = c * nx + sn * ny;
                vt1 = c * ny - sn * nx;
            }
            double vz1 = nz;
            int fate = 0;
            if (z1 < 0.0) {
                if (p->wall_bc[0] == 1) { z1 = -z1; vz1 = -vz1; }
                else fate = (r1 < p->cathode_rmax) ? 1 : 2;
            }
            if (fate == 0 && r1 >= R) {
                if (p->wall_bc[2] == 1) { r1 = 2.0 * R - r1; vr1 = -vr1; if (r1 >= R) r1 = nextafter(R, 0.0); }
                else fate = 3;
            }
            if (fate == 0 && z1 >= L) {
                if (p->wall_bc[1] == 1) { z1 = 2.0 * L - z1; vz1 = -vz1; if (z1 >= L) z1 = nextafter(L, 0.0); }
                else fate = 4;
            }
            S->r[k] = r1; S->z[k] = z1; S->vr[k] = vr1; S->vt[k] = vt1; S->vz[k] = vz1;
            if (fate) {
                dead[s][k] = 1;
                a->n_abs[fate]++;
                if (fate == 1) {
                    a->dq += p->q[s] * p->w[s];
                    if (s == 1 && p->ied_hist && r1 >= p->ied_r0 && r1 < p->ied_r1) {
                        const double e_ev = 0.5 * p->m[1] * (vr1 * vr1 + vt1 * vt1 + vz1 * vz1) / QE;
                        double x = floor(e_ev / p->ied_emax * p->ied_nbins);
                        const int64_t b = (x >= p->ied_nbins) ? p->ied_nbins : (int64_t)x;
#ifdef _OPENMP
#pragma omp atomic
#endif
                        p->ied_hist[b]++;
                    }
                    /* secondary emission (Section 3): ions with yield
                     * gamma_i, electrons with gamma_e, independently; the
                     * secondary is an electron at rest at (r', 0) */
                    if (p->see_on && t_see[s] > 0) {
                        uint32_t u[4];
                        draw(p, S->id[k], s, PUR_SEE, st->step, u);
                        if ((uint64_t)u[0] < t_see[s]) {
                            child c = {child_key(s, S->id[k], 0), 0, r1, 0.0, 0.0, 0.0, 0.0};
                            push_child(&a->kids, c);
                            a->dq -= p->q[0] * p->w[0];
                            if (s == 1) a->n_see++;
                            else a->n_see_e++;
                        }
                    }
                }
            }
        }
        /* combine the threads' results in thread order */
        dq = 0.0;
        for (int t = 0; t < nthr; ++t) {
            d->ke[s] += acc[t].ke;
            d->pz[s] += acc[t].pz;
            dq += acc[t].dq;
            for (int f = 0; f < 5; ++f) { d->n_abs[s][f] += acc[t].n_abs[f]; acc[t].n_abs[f] = 0; }
            d->n_see += acc[t].n_see;
            d->n_see_e += acc[t].n_see_e;
            acc[t].n_see = acc[t].n_see_e = 0;
            append_children(&kids, &acc[t].kids);
        }
    }

    /* MCC for electrons that existed before the step and are still inside. */
    if (p->mcc_on) {
        orc_species *S = &sp[0];
        const double me = p->m[0];
        const int64_t ne = n_pre[0];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t k = 0; k < ne; ++k) {
            thread_acc *a = &acc[orc_thread_id()];
            if (dead[0][k]) continue;
            double vx = S->vr[k], vy = S->vt[k], vz = S->vz[k];
            int proc = orc_mcc_select(p, nu, numax, t_null, S->id[k], st->step, vx, vy, vz, NULL);
            if (proc == -2) continue;
            a->n_cand++;
            if (proc < 0) continue;
            a->n_coll[proc]++;
            uint32_t u[4];
            draw(p, S->id[k], 0, PUR_MCC, st->step, u);
            double v2 = vx * vx + vy * vy + vz * vz;
            double e = 0.5 * me * v2 / QE;
            double dn[3];
            iso_dir(u[2], u[3], dn);
            double enew;
            if (proc == 0) {
                /* elastic: E' = E (1 - (2 m_e / M)(1 - cos theta)) */
                double vm = sqrt(v2);
                double cth = (vx * dn[0] + vy * dn[1] + vz * dn[2]) / vm;
                enew = e * (1.0 - 2.0 * me / p->m[1] * (1.0 - cth));
            } else if (proc == 1) {
                enew = e - p->e_exc;
            } else {
                /* ionization from the ground state (2) or from the metastable
                 * (3): the remaining energy is split uniformly between the
                 * scattered and the ejected electron; a new ion with the gas
                 * temperature appears at the same place. */
                double erem = e - ((proc == 2) ? p->e_iz : p->e_iz_meta);
                uint32_t ua[4], ub[4];
                draw(p, S->id[k], 0, PUR_IZ, st->step, ua);
                draw(p, S->id[k], 0, PUR_ION, st->step, ub);
                double eej = u24(ua[0]) * erem;
                enew = (1.0 - u24(ua[0])) * erem;   /* = erem - eej, without cancellation */
                double de_[3];
                iso_dir(ua[1], ua[2], de_);
                double vej = sqrt(2.0 * QE * eej / me);
                child ce = {child_key(0, S->id[k], 0), 0, S->r[k], S->z[k],
                            vej * de_[0], vej * de_[1], vej * de_[2]};
                push_child(&a->kids, ce);
                double sig = sqrt(KB * p->t_gas / p->m[1]);
                double a0 = sqrt(-2.0 * log(u_open(ub[0]))), p0 = 2.0 * PI * u24(ub[1]);
                double a1 = sqrt(-2.0 * log(u_open(ub[2]))), p1 = 2.0 * PI * u24(ub[3]);
                child ci = {child_key(0, S->id[k], 1), 1, S->r[k], S->z[k],
                            sig * a0 * cos(p0), sig * a0 * sin(p0), sig * a1 * cos(p1)};
                push_child(&a->kids, ci);
            }
            double vnew = sqrt(2.0 * QE * enew / me);
            S->vr[k] = vnew * dn[0];
            S->vt[k] = vnew * dn[1];
            S->vz[k] = vnew * dn[2];
        }
        for (int t = 0; t < nthr; ++t) {
            d->n_cand += acc[t].n_cand;
            for (int c = 0; c < 4; ++c) d->n_coll[c] += acc[t].n_coll[c];
            append_children(&kids, &acc[t].kids);
        }
    }
    free(acc);

    /* remove absorbed particles, keeping order */
    for (int s = 0; s < 2; ++s) {
        orc_species *S = &sp[s];
        int64_t w = 0;
        for (int64_t k = 0; k < n_pre[s]; ++k) {
            if (dead[s][k]) continue;
            S->r[w] = S->r[k]; S->z[w] = S->z[k];
            S->vr[w] = S->vr[k]; S->vt[w] = S->vt[k]; S->vz[w] = S->vz[k];
            S->id[w] = S->id[k];
            ++w;
        }
        S->n = w;
        free(dead[s]);
    }
    /* new particles: ids in (parent species, parent id, kind) order */
    qsort(kids.a, kids.n, sizeof(child), child_cmp);
    for (int64_t c = 0; c < kids.n; ++c) {
        const child *k = &kids.a[c];
        orc_species *S = &sp[k->species];
        if (S->n >= S->cap) { rc = -2; continue; }
        int64_t w = S->n++;
        S->r[w] = k->r; S->z[w] = k->z;
        S->vr[w] = k->vr; S->vt[w] = k->vt; S->vz[w] = k->vz;
        S->id[w] = st->next_id[k->species]++;
        d->n_child[k->species]++;
    }
    free(kids.a);

    /* deposit */
    deposit_all(p, sp, q_e, q_i);
    for (int64_t n = 0; n < nn; ++n) { d->q_dep[0] += q_e[n]; d->q_dep[1] += q_i[n]; }
    {
        /* peak density of each species: node charge over (q_s times the node volume) */
        double *vol = malloc(sizeof(double) * nn);
        orc_node_volumes(p, vol);
        d->n_peak[0] = d->n_peak[1] = -HUGE_VAL;
        for (int64_t n = 0; n < nn; ++n) {
            d->n_peak[0] = fmax(d->n_peak[0], q_e[n] / (p->q[0] * vol[n]));
            d->n_peak[1] = fmax(d->n_peak[1], q_i[n] / (p->q[1] * vol[n]));
        }
        free(vol);
    }

    /* field solve and circuit */
    d->dq_conv = dq;
    if (p->field_solve) {
        double *qt = malloc(sizeof(double) * nn);
        for (int64_t n = 0; n < nn; ++n) qt[n] = q_e[n] + q_i[n];
        if (orc_solve(p, qt, 0.0, phi0, p->poisson_rtol, p->poisson_maxit,
                      &d->poisson_iters, &d->poisson_res)) rc = rc ? rc : -4;
        double qc0 = orc_induced_charge(p, phi0, qt);
        d->qc0 = qc0;
        double v;
        if (p->circuit == 1)
            v = (st->qc + dq + dt * p->v_ext / p->r_ext - qc0) / (st->cap_c + dt / p->r_ext);
        else
            v = p->v_fixed;
        st->vc = v;
        st->qc = qc0 + st->cap_c * v;
        for (int64_t n = 0; n < nn; ++n) phi[n] = phi0[n] + v * phi_l[n];
        free(qt);
    }
    d->i_cathode = dq / dt;
    d->phi_max = -HUGE_VAL;
    for (int64_t n = 0; n < nn; ++n) d->phi_max = fmax(d->phi_max, phi[n]);
    st->step++;
    free(ern); free(ezn); free(nu);
    return rc;
}
