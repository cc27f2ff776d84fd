/*
 * SDC sweeps, the FAS coupling of two levels and serial PFASST for the
 * oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Time slices are emulated in one process: the values a time rank would
 * send forward are taken from explicit snapshots, so the result is what P
 * ranks running the algorithm in lock step would compute.
 *
 * Readings of the paper used here (it defers the algorithm's detail to
 * companion papers):
 *  - one sweep per level per iteration; the fine rank's new initial value
 *    is the previous slice's end value after the previous iteration;
 *  - the predictor is pipelined: in round j every slice p >= j takes the
 *    end value of slice p-1 from round j-1 and does one coarse sweep;
 *  - FAS term in integral form: tau = R(dt Q_f F_f) - dt Q_c F_c(R U_f),
 *    which keeps R of the fine collocation solution a coarse fixed point;
 *  - restriction is point-wise injection in space and in time (the coarse
 *    nodes are a subset of the fine nodes); interpolation is d-linear in
 *    space and Lagrange in time over the coarse nodes;
 *  - F at node 0 is recomputed whenever node 0 changes;
 *  - the V-cycle initial guess is the previous iterate at the same node;
 *  - options (the paper leaves both open): with f_solve, F at a node after
 *    its solve is (U - b) / (dt d_m), what the implicit-Euler substep
 *    implies, equal to nu L U when the solve is exact; with f_interp, the
 *    fine F values take the interpolated coarse F correction instead of
 *    being re-evaluated on the corrected U.  With either, the stored F is
 *    no longer F(U) until the iteration converges, so the collocation
 *    residual re-evaluates F(U).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

struct or_pfasst {
    or_params p;
    int nl;                  /* levels: 1 (single) or 2 */
    int n[2], nn[2];         /* grid size, number of nodes */
    size_t len[2];           /* points per field */
    double s[2][16], Q[2][256], S[2][256], d[2][16];
    double Lt[16 * 16];      /* fine node x coarse node */
    int cmap[16];            /* coarse node -> coarse-coinciding fine node */
    double *U[2], *F[2];     /* [P][nn][len] */
    double *tau, *Uold;      /* coarse: [P][nn_c][len_c] */
    double *Fold;            /* coarse F at restriction (f_interp) */
    double *ublock, *ublock_c;
    long long vcyc[2];
};

static size_t glen(int dim, int n)
{
    size_t l = 1;
    for (int d = 0; d < dim; ++d) l *= (size_t)n;
    return l;
}

static double *fld(or_pfasst *c, double *base, int lev, int p, int m)
{
    return base + ((size_t)p * c->nn[lev] + (size_t)m) * c->len[lev];
}

double *or_pfasst_field(or_pfasst *c, int which, int p, int m)
{
    switch (which) {
    case OR_UF: return fld(c, c->U[0], 0, p, m);
    case OR_FF: return fld(c, c->F[0], 0, p, m);
    case OR_UC: return c->nl > 1 ? fld(c, c->U[1], 1, p, m) : NULL;
    case OR_FC: return c->nl > 1 ? fld(c, c->F[1], 1, p, m) : NULL;
    case OR_TAU: return c->nl > 1 ? fld(c, c->tau, 1, p, m) : NULL;
    case OR_UCOLD: return c->nl > 1 ? fld(c, c->Uold, 1, p, m) : NULL;
    case OR_FCOLD: return c->nl > 1 && c->Fold ? fld(c, c->Fold, 1, p, m) : NULL;
    }
    return NULL;
}

long long or_pfasst_vcycles(or_pfasst *c, int level) { return c->vcyc[level]; }

void or_pfasst_matrices(or_pfasst *c, int level, double *s, double *Q)
{
    int nn = c->nn[level];
    memcpy(s, c->s[level], nn * sizeof(double));
    memcpy(Q, c->Q[level], nn * nn * sizeof(double));
}

or_pfasst *or_pfasst_create(const or_params *prm)
{
    if (prm->dim < 1 || prm->dim > 3 || prm->n < 1 || prm->n_slices < 1) return NULL;
    if (prm->nodes_fine < 2 || prm->nodes_fine > 16) return NULL;
    if (prm->node_family != OR_NODES_LOBATTO && prm->node_family != OR_NODES_UNIFORM) return NULL;
    if (prm->stencil_order != 2 && prm->stencil_order != 4) return NULL;
    if (prm->stencil_order == 4 && prm->mg.mixed) return NULL;
    if ((prm->f_solve != 0 && prm->f_solve != 1) || (prm->f_interp != 0 && prm->f_interp != 1)) return NULL;
    if (prm->residual_abs != 0 && prm->residual_abs != 1) return NULL;
    or_pfasst *c = (or_pfasst *)calloc(1, sizeof(or_pfasst));
    c->p = *prm;
    c->nl = prm->nodes_coarse > 0 ? 2 : 1;
    c->n[0] = prm->n;
    c->nn[0] = prm->nodes_fine;
    if (c->nl > 1) {
        if ((prm->n & 1) == 0 || prm->n < 3) { free(c); return NULL; }
        c->n[1] = (prm->n + 1) / 2 - 1;
        c->nn[1] = prm->nodes_coarse;
    }
    for (int l = 0; l < c->nl; ++l) {
        c->len[l] = glen(prm->dim, c->n[l]);
        if (prm->node_family == OR_NODES_UNIFORM) or_uniform_nodes(c->nn[l], c->s[l]);
        else or_lobatto_nodes(c->nn[l], c->s[l]);
        or_qmat_family(c->nn[l], c->s[l], prm->node_family, c->Q[l], c->S[l], c->d[l]);
        size_t tot = (size_t)prm->n_slices * c->nn[l] * c->len[l];
        c->U[l] = (double *)calloc(tot, sizeof(double));
        c->F[l] = (double *)calloc(tot, sizeof(double));
    }
    c->ublock = (double *)calloc(c->len[0], sizeof(double));
    if (c->nl > 1) {
        size_t tot = (size_t)prm->n_slices * c->nn[1] * c->len[1];
        c->tau = (double *)calloc(tot, sizeof(double));
        c->Uold = (double *)calloc(tot, sizeof(double));
        if (prm->f_interp) c->Fold = (double *)calloc(tot, sizeof(double));
        c->ublock_c = (double *)calloc(c->len[1], sizeof(double));
        or_interp_matrix(c->nn[0], c->s[0], c->nn[1], c->s[1], c->Lt);
        for (int mc = 0; mc < c->nn[1]; ++mc) {
            c->cmap[mc] = -1;
            for (int mf = 0; mf < c->nn[0]; ++mf)
                if (fabs(c->s[0][mf] - c->s[1][mc]) < 1e-14) c->cmap[mc] = mf;
            if (c->cmap[mc] < 0) { or_pfasst_destroy(c); return NULL; }
        }
    }
    return c;
}

void or_pfasst_destroy(or_pfasst *c)
{
    if (!c) return;
    for (int l = 0; l < 2; ++l) { free(c->U[l]); free(c->F[l]); }
    free(c->tau);
    free(c->Uold);
    free(c->Fold);
    free(c->ublock);
    free(c->ublock_c);
    free(c);
}

/* F = nu L_h u on level lev (the fine level's L is fourth order when
 * stencil_order is 4). */
static void feval(or_pfasst *c, int lev, const double *u, double *f)
{
    if (lev == 0 && c->p.stencil_order == 4) or_lap4(c->p.dim, c->n[lev], u, f);
    else or_lap(c->p.dim, c->n[lev], u, f);
    const size_t len = c->len[lev];
    for (size_t x = 0; x < len; ++x) f[x] = c->p.nu * f[x];
}

/* Point-wise injection: coarse 1-based J <- fine 1-based 2J. */
static void inject(int dim, int nf, const double *uf, double *uc)
{
    const int nc = (nf + 1) / 2 - 1;
    const int ncy = dim >= 2 ? nc : 1, ncz = dim >= 3 ? nc : 1;
    for (int K = 0; K < ncz; ++K)
        for (int J = 0; J < ncy; ++J)
            for (int I = 0; I < nc; ++I) {
                size_t fi = 2 * I + 1, fj = dim >= 2 ? 2 * J + 1 : 0, fk = dim >= 3 ? 2 * K + 1 : 0;
                uc[I + (size_t)nc * (J + (size_t)nc * K)] = uf[fi + (size_t)nf * (fj + (size_t)nf * fk)];
            }
}

/* One SDC sweep with backward-Euler substeps (eq. sdc-be with the
 * integrals of the old function values, written for the linear problem as
 * in eq. SDCcompactLIII): for m = 0..M-1
 *   b = U[m] - dt_{m+1} F^k[m+1] + I_m (+ tau[m+1] - tau[m] on level 1),
 *   solve (I - nu dt_{m+1} L) U[m+1] = b from U^k[m+1], F[m+1] = nu L U[m+1]
 *   (f_solve: F[m+1] = (U[m+1] - b) / dt_{m+1}). */
void or_sdc_sweep(or_pfasst *c, int lev, int p)
{
    const int nn = c->nn[lev], M = nn - 1;
    const size_t len = c->len[lev];
    const double dt = c->p.dt;
    double *I = (double *)malloc((size_t)M * len * sizeof(double));
    double *b = (double *)malloc(len * sizeof(double));
    for (int m = 0; m < M; ++m) {
        double *Im = I + (size_t)m * len;
#pragma omp parallel for schedule(static) if (len > 65536)
        for (size_t x = 0; x < len; ++x) {
            double acc = 0.0;
            for (int i = 0; i < nn; ++i) acc += c->S[lev][m * nn + i] * fld(c, c->F[lev], lev, p, i)[x];
            Im[x] = dt * acc;
        }
    }
    for (int m = 0; m < M; ++m) {
        const double dtm = dt * c->d[lev][m + 1];
        const double *Um = fld(c, c->U[lev], lev, p, m);
        const double *Fm1 = fld(c, c->F[lev], lev, p, m + 1);
        const double *Im = I + (size_t)m * len;
#pragma omp parallel for schedule(static) if (len > 65536)
        for (size_t x = 0; x < len; ++x) b[x] = Um[x] - dtm * Fm1[x] + Im[x];
        if (lev == 1) {
            const double *t1 = fld(c, c->tau, 1, p, m + 1), *t0 = fld(c, c->tau, 1, p, m);
            for (size_t x = 0; x < len; ++x) b[x] = b[x] + (t1[x] - t0[x]);
        }
        double *u = fld(c, c->U[lev], lev, p, m + 1);
        if (lev == 0 && c->p.stencil_order == 4)
            c->vcyc[lev] += or_mg_solve4(c->p.dim, c->n[lev], c->p.nu * dtm, &c->p.mg, b, u, NULL);
        else
            c->vcyc[lev] += or_mg_solve(c->p.dim, c->n[lev], c->p.nu * dtm, &c->p.mg, b, u, NULL);
        double *fm = fld(c, c->F[lev], lev, p, m + 1);
        if (c->p.f_solve)
            for (size_t x = 0; x < len; ++x) fm[x] = (u[x] - b[x]) / dtm;
        else feval(c, lev, u, fm);
    }
    free(I);
    free(b);
}

/* FAS restriction of slice p (Sec. 2.3): U_c = R U_f, F_c = nu L_2h U_c,
 * tau = R(dt Q_f F_f) - dt Q_c F_c; the restricted state is kept as U_c^old. */
void or_fas_restrict(or_pfasst *c, int p)
{
    const int dim = c->p.dim, nf = c->n[0], nnf = c->nn[0], nnc = c->nn[1];
    const size_t lf = c->len[0], lc = c->len[1];
    const double dt = c->p.dt;
    for (int mc = 0; mc < nnc; ++mc) {
        double *uc = fld(c, c->U[1], 1, p, mc);
        inject(dim, nf, fld(c, c->U[0], 0, p, c->cmap[mc]), uc);
        feval(c, 1, uc, fld(c, c->F[1], 1, p, mc));
    }
    double *qf = (double *)malloc(lf * sizeof(double));
    double *qfc = (double *)malloc(lc * sizeof(double));
    for (int mc = 0; mc < nnc; ++mc) {
        const int mf = c->cmap[mc];
#pragma omp parallel for schedule(static) if (lf > 65536)
        for (size_t x = 0; x < lf; ++x) {
            double acc = 0.0;
            for (int i = 0; i < nnf; ++i) acc += c->Q[0][mf * nnf + i] * fld(c, c->F[0], 0, p, i)[x];
            qf[x] = dt * acc;
        }
        inject(dim, nf, qf, qfc);
        double *t = fld(c, c->tau, 1, p, mc);
        for (size_t x = 0; x < lc; ++x) {
            double acc = 0.0;
            for (int j = 0; j < nnc; ++j) acc += c->Q[1][mc * nnc + j] * fld(c, c->F[1], 1, p, j)[x];
            t[x] = qfc[x] - dt * acc;
        }
    }
    memcpy(fld(c, c->Uold, 1, p, 0), fld(c, c->U[1], 1, p, 0), (size_t)nnc * lc * sizeof(double));
    if (c->Fold) memcpy(fld(c, c->Fold, 1, p, 0), fld(c, c->F[1], 1, p, 0), (size_t)nnc * lc * sizeof(double));
    free(qf);
    free(qfc);
}

/* Interpolation of slice p: U_f[m] += P_s sum_mc L_t[m][mc] (U_c - U_c^old)[mc]
 * for every fine node, then F_f recomputed (f_interp: F_f[m] += P_s sum_mc
 * L_t[m][mc] (F_c - F_c^old)[mc], the same interpolation of the coarse F
 * change). */
void or_interpolate(or_pfasst *c, int p)
{
    const int dim = c->p.dim, nc = c->n[1], nnf = c->nn[0], nnc = c->nn[1];
    const size_t lc = c->len[1];
    double *dc = (double *)malloc(lc * sizeof(double));
    for (int m = 0; m < nnf; ++m) {
#pragma omp parallel for schedule(static) if (lc > 65536)
        for (size_t x = 0; x < lc; ++x) {
            double acc = 0.0;
            for (int mc = 0; mc < nnc; ++mc)
                acc += c->Lt[m * nnc + mc] * (fld(c, c->U[1], 1, p, mc)[x] - fld(c, c->Uold, 1, p, mc)[x]);
            dc[x] = acc;
        }
        double *uf = fld(c, c->U[0], 0, p, m);
        if (c->p.interp_order == 4 && nc >= 3) or_prolong4_add(dim, nc, dc, uf);
        else or_prolong_add(dim, nc, dc, uf);
        double *ff = fld(c, c->F[0], 0, p, m);
        if (!c->p.f_interp) {
            feval(c, 0, uf, ff);
            continue;
        }
        for (size_t x = 0; x < lc; ++x) {
            double acc = 0.0;
            for (int mc = 0; mc < nnc; ++mc)
                acc += c->Lt[m * nnc + mc] * (fld(c, c->F[1], 1, p, mc)[x] - fld(c, c->Fold, 1, p, mc)[x]);
            dc[x] = acc;
        }
        if (c->p.interp_order == 4 && nc >= 3) or_prolong4_add(dim, nc, dc, ff);
        else or_prolong_add(dim, nc, dc, ff);
    }
    free(dc);
}

void or_pfasst_spread(or_pfasst *c, const double *u_block)
{
    const int P = c->p.n_slices;
    memcpy(c->ublock, u_block, c->len[0] * sizeof(double));
    for (int p = 0; p < P; ++p)
        for (int m = 0; m < c->nn[0]; ++m) {
            memcpy(fld(c, c->U[0], 0, p, m), u_block, c->len[0] * sizeof(double));
            feval(c, 0, u_block, fld(c, c->F[0], 0, p, m));
        }
    if (c->nl > 1) inject(c->p.dim, c->n[0], u_block, c->ublock_c);
}

/* Predictor (Sec. 2.4): rounds j = 0..P-1; in round j every slice p >= j
 * (for j >= 1) takes the coarse end value slice p-1 had after round j-1
 * and does one coarse sweep, so slice p sweeps p+1 times. */
void or_pfasst_predictor(or_pfasst *c)
{
    if (c->nl < 2) return;
    const int P = c->p.n_slices, Mc = c->nn[1] - 1;
    const size_t lc = c->len[1];
    for (int p = 0; p < P; ++p) or_fas_restrict(c, p);
    double *E = (double *)malloc((size_t)P * lc * sizeof(double));
    for (int j = 0; j < P; ++j) {
        for (int p = 0; p < P; ++p) memcpy(E + p * lc, fld(c, c->U[1], 1, p, Mc), lc * sizeof(double));
        for (int p = j; p < P; ++p) {
            if (j >= 1 && p >= 1) {
                double *u0 = fld(c, c->U[1], 1, p, 0);
                memcpy(u0, E + (size_t)(p - 1) * lc, lc * sizeof(double));
                feval(c, 1, u0, fld(c, c->F[1], 1, p, 0));
            }
            or_sdc_sweep(c, 1, p);
        }
    }
    free(E);
    for (int p = 0; p < P; ++p) or_interpolate(c, p);
}

/* Collocation residual (eq. resid) per slice:
 *   r[m] = U0_p - U[m] + dt sum_i Q[m][i] F(U[i]),  m = 0..M,
 * with U0_p the previous slice's end value (u_block for p = 0), normalised
 * by |U0_p|_inf (residual_abs: not normalised); the block residual is the
 * maximum over slices.  The stored
 * F are F(U) unless f_solve or f_interp is set; then F(U) is re-evaluated. */
double or_pfasst_residual(or_pfasst *c, double *res)
{
    const int P = c->p.n_slices, nn = c->nn[0], M = nn - 1;
    const size_t len = c->len[0];
    const double dt = c->p.dt;
    const int reeval = c->p.f_solve || c->p.f_interp;
    double *Fe = reeval ? (double *)malloc((size_t)nn * len * sizeof(double)) : NULL;
    double blk = 0.0;
    for (int p = 0; p < P; ++p) {
        const double *Fp = fld(c, c->F[0], 0, p, 0);
        if (reeval) {
            for (int i = 0; i < nn; ++i) feval(c, 0, fld(c, c->U[0], 0, p, i), Fe + (size_t)i * len);
            Fp = Fe;
        }
        const double *u0 = p == 0 ? c->ublock : fld(c, c->U[0], 0, p - 1, M);
        double rmax = 0.0;
        for (int m = 0; m <= M; ++m) {
            const double *um = fld(c, c->U[0], 0, p, m);
            for (size_t x = 0; x < len; ++x) {
                double acc = 0.0;
                for (int i = 0; i < nn; ++i) acc += c->Q[0][m * nn + i] * Fp[(size_t)i * len + x];
                double r = fabs(u0[x] - um[x] + dt * acc);
                if (r > rmax || r != r) rmax = r;
            }
        }
        double n0 = or_norm_inf(len, u0);
        double rp = c->p.residual_abs ? rmax : (n0 > 0 ? rmax / n0 : rmax);
        if (res) res[p] = rp;
        if (rp > blk || rp != rp) blk = rp;
    }
    free(Fe);
    return blk;
}

/* One iteration (Sec. 2.4): new fine initial values from the previous
 * slice, fine sweeps, FAS restriction, the coarse sweeps in slice order,
 * interpolation, residual.  With one level: initial values and sweeps. */
double or_pfasst_iter(or_pfasst *c)
{
    const int P = c->p.n_slices, Mf = c->nn[0] - 1;
    const size_t lf = c->len[0];
    double *E = (double *)malloc((size_t)P * lf * sizeof(double));
    for (int p = 0; p < P; ++p) memcpy(E + p * lf, fld(c, c->U[0], 0, p, Mf), lf * sizeof(double));
    for (int p = 1; p < P; ++p) {
        double *u0 = fld(c, c->U[0], 0, p, 0);
        memcpy(u0, E + (size_t)(p - 1) * lf, lf * sizeof(double));
        feval(c, 0, u0, fld(c, c->F[0], 0, p, 0));
    }
    free(E);
    for (int p = 0; p < P; ++p) or_sdc_sweep(c, 0, p);
    if (c->nl > 1) {
        const int Mc = c->nn[1] - 1;
        const size_t lc = c->len[1];
        for (int p = 0; p < P; ++p) or_fas_restrict(c, p);
        for (int p = 0; p < P; ++p) {
            double *u0 = fld(c, c->U[1], 1, p, 0);
            memcpy(u0, p == 0 ? c->ublock_c : fld(c, c->U[1], 1, p - 1, Mc), lc * sizeof(double));
            feval(c, 1, u0, fld(c, c->F[1], 1, p, 0));
            or_sdc_sweep(c, 1, p);
        }
        for (int p = 0; p < P; ++p) or_interpolate(c, p);
    }
    return or_pfasst_residual(c, NULL);
}
