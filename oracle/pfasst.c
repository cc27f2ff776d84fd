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
 *  - fine_send = 1: the fine end value a slice sends is the one right after
 *    its fine sweep (before the coarse correction reaches it), taken up by
 *    the next slice at its next iteration; before the first iteration it is
 *    the end value the predictor leaves;
 *  - the V-cycle initial guess is the previous iterate at the same node;
 *  - three levels (nodes_middle > 0; Sec. 4.2's weak-scaling runs): the
 *    FAS term of a level below the middle one carries the finer level's
 *    own term through the restriction, tau_c = R(dt Q_f F_f + tau_f) -
 *    dt Q_c F_c(R U_f); an iteration sweeps the fine level, restricts,
 *    sweeps the middle level, restricts, runs the coarse chain, interpolates
 *    to the middle level, sweeps it again and interpolates to the fine
 *    level; the middle level's node 0 is what the restriction and the
 *    interpolation of the coarse correction leave there (no separate
 *    send-forward); the predictor interpolates straight up without
 *    middle-level sweeps;
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
    int nl;                  /* levels: 1 (single), 2 or 3 */
    int n[3], nn[3];         /* grid size, number of nodes */
    size_t len[3];           /* points per field */
    double s[3][16], Q[3][256], S[3][256], d[3][16];
    double Lt[2][16 * 16];   /* level l node x level l+1 node */
    int cmap[2][16];         /* level l+1 node -> coinciding level l node */
    double *U[3], *F[3];     /* [P][nn][len] */
    double *tau[3], *Uold[3];/* levels >= 1: [P][nn][len] */
    double *Fold[3];         /* levels >= 1: F at restriction (f_interp) */
    double *ub[3];           /* the block's initial value on each level */
    double *Esnap;           /* fine_send = 1: [P][len0] end values after the fine sweep */
    double *ublock;          /* = ub[0] */
    long long vcyc[3];
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
    case OR_TAU: return c->nl > 1 ? fld(c, c->tau[1], 1, p, m) : NULL;
    case OR_UCOLD: return c->nl > 1 ? fld(c, c->Uold[1], 1, p, m) : NULL;
    case OR_FCOLD: return c->nl > 1 && c->Fold[1] ? fld(c, c->Fold[1], 1, p, m) : NULL;
    }
    return NULL;
}

double *or_pfasst_level_field(or_pfasst *c, int lev, int kind, int p, int m)
{
    if (lev < 0 || lev >= c->nl || p < 0 || p >= c->p.n_slices || m < 0 || m >= c->nn[lev]) return NULL;
    switch (kind) {
    case OR_K_U: return fld(c, c->U[lev], lev, p, m);
    case OR_K_F: return fld(c, c->F[lev], lev, p, m);
    case OR_K_TAU: return lev > 0 ? fld(c, c->tau[lev], lev, p, m) : NULL;
    case OR_K_UOLD: return lev > 0 ? fld(c, c->Uold[lev], lev, p, m) : NULL;
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
    if (prm->nodes_middle != 0 && (prm->nodes_coarse == 0 || prm->nodes_middle < 2 || prm->nodes_middle > 16))
        return NULL;
    if (prm->fine_send != 0 && prm->fine_send != 1) return NULL;
    or_pfasst *c = (or_pfasst *)calloc(1, sizeof(or_pfasst));
    c->p = *prm;
    c->nl = prm->nodes_coarse == 0 ? 1 : prm->nodes_middle > 0 ? 3 : 2;
    c->n[0] = prm->n;
    c->nn[0] = prm->nodes_fine;
    if (c->nl == 2) c->nn[1] = prm->nodes_coarse;
    if (c->nl == 3) {
        c->nn[1] = prm->nodes_middle;
        c->nn[2] = prm->nodes_coarse;
    }
    for (int l = 1; l < c->nl; ++l) {
        if ((c->n[l - 1] & 1) == 0 || c->n[l - 1] < 3) { free(c); return NULL; }
        c->n[l] = (c->n[l - 1] + 1) / 2 - 1;
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
    for (int l = 0; l < c->nl; ++l) c->ub[l] = (double *)calloc(c->len[l], sizeof(double));
    c->ublock = c->ub[0];
    if (prm->fine_send) c->Esnap = (double *)calloc((size_t)prm->n_slices * c->len[0], sizeof(double));
    for (int l = 1; l < c->nl; ++l) {
        size_t tot = (size_t)prm->n_slices * c->nn[l] * c->len[l];
        c->tau[l] = (double *)calloc(tot, sizeof(double));
        c->Uold[l] = (double *)calloc(tot, sizeof(double));
        if (prm->f_interp) c->Fold[l] = (double *)calloc(tot, sizeof(double));
        or_interp_matrix(c->nn[l - 1], c->s[l - 1], c->nn[l], c->s[l], c->Lt[l - 1]);
        for (int mc = 0; mc < c->nn[l]; ++mc) {
            c->cmap[l - 1][mc] = -1;
            for (int mf = 0; mf < c->nn[l - 1]; ++mf)
                if (fabs(c->s[l - 1][mf] - c->s[l][mc]) < 1e-14) c->cmap[l - 1][mc] = mf;
            if (c->cmap[l - 1][mc] < 0) { or_pfasst_destroy(c); return NULL; }
        }
    }
    return c;
}

void or_pfasst_destroy(or_pfasst *c)
{
    if (!c) return;
    for (int l = 0; l < 3; ++l) {
        free(c->U[l]);
        free(c->F[l]);
        free(c->tau[l]);
        free(c->Uold[l]);
        free(c->Fold[l]);
        free(c->ub[l]);
    }
    free(c->Esnap);
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
        if (lev >= 1) {
            const double *t1 = fld(c, c->tau[lev], lev, p, m + 1), *t0 = fld(c, c->tau[lev], lev, p, m);
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

/* FAS restriction of slice p from level l to level l+1 (Sec. 2.3):
 * U_c = R U_f, F_c = nu L U_c, tau_c = R(dt Q_f F_f + tau_f) - dt Q_c F_c
 * (tau_f = 0 on the fine level); the restricted state is kept as U_c^old
 * (and F_c as F_c^old with f_interp). */
void or_fas_restrict_level(or_pfasst *c, int l, int p)
{
    const int L = l + 1;
    const int dim = c->p.dim, nf = c->n[l], nnf = c->nn[l], nnc = c->nn[L];
    const size_t lf = c->len[l], lc = c->len[L];
    const double dt = c->p.dt;
    for (int mc = 0; mc < nnc; ++mc) {
        double *uc = fld(c, c->U[L], L, p, mc);
        inject(dim, nf, fld(c, c->U[l], l, p, c->cmap[l][mc]), uc);
        feval(c, L, uc, fld(c, c->F[L], L, p, mc));
    }
    double *qf = (double *)malloc(lf * sizeof(double));
    double *qfc = (double *)malloc(lc * sizeof(double));
    for (int mc = 0; mc < nnc; ++mc) {
        const int mf = c->cmap[l][mc];
        const double *tf = l > 0 ? fld(c, c->tau[l], l, p, mf) : NULL;
#pragma omp parallel for schedule(static) if (lf > 65536)
        for (size_t x = 0; x < lf; ++x) {
            double acc = 0.0;
            for (int i = 0; i < nnf; ++i) acc += c->Q[l][mf * nnf + i] * fld(c, c->F[l], l, p, i)[x];
            qf[x] = tf ? dt * acc + tf[x] : dt * acc;
        }
        inject(dim, nf, qf, qfc);
        double *t = fld(c, c->tau[L], L, p, mc);
        for (size_t x = 0; x < lc; ++x) {
            double acc = 0.0;
            for (int j = 0; j < nnc; ++j) acc += c->Q[L][mc * nnc + j] * fld(c, c->F[L], L, p, j)[x];
            t[x] = qfc[x] - dt * acc;
        }
    }
    memcpy(fld(c, c->Uold[L], L, p, 0), fld(c, c->U[L], L, p, 0), (size_t)nnc * lc * sizeof(double));
    if (c->Fold[L]) memcpy(fld(c, c->Fold[L], L, p, 0), fld(c, c->F[L], L, p, 0), (size_t)nnc * lc * sizeof(double));
    free(qf);
    free(qfc);
}

void or_fas_restrict(or_pfasst *c, int p) { or_fas_restrict_level(c, 0, p); }

/* Interpolation of slice p from level l+1 to level l: U_l[m] += P_s sum_mc
 * L_t[m][mc] (U_{l+1} - U_{l+1}^old)[mc] for every node m of level l, then
 * F_l recomputed (f_interp: F_l[m] += P_s sum_mc L_t[m][mc] (F_{l+1} -
 * F_{l+1}^old)[mc], the same interpolation of the coarse F change). */
void or_interpolate_level(or_pfasst *c, int l, int p)
{
    const int L = l + 1;
    const int dim = c->p.dim, nc = c->n[L], nnf = c->nn[l], nnc = c->nn[L];
    const size_t lc = c->len[L];
    const double *Lt = c->Lt[l];
    double *dc = (double *)malloc(lc * sizeof(double));
    for (int m = 0; m < nnf; ++m) {
#pragma omp parallel for schedule(static) if (lc > 65536)
        for (size_t x = 0; x < lc; ++x) {
            double acc = 0.0;
            for (int mc = 0; mc < nnc; ++mc)
                acc += Lt[m * nnc + mc] * (fld(c, c->U[L], L, p, mc)[x] - fld(c, c->Uold[L], L, p, mc)[x]);
            dc[x] = acc;
        }
        double *uf = fld(c, c->U[l], l, p, m);
        if (c->p.interp_order == 4 && nc >= 3) or_prolong4_add(dim, nc, dc, uf);
        else or_prolong_add(dim, nc, dc, uf);
        double *ff = fld(c, c->F[l], l, p, m);
        if (!c->p.f_interp) {
            feval(c, l, uf, ff);
            continue;
        }
        for (size_t x = 0; x < lc; ++x) {
            double acc = 0.0;
            for (int mc = 0; mc < nnc; ++mc)
                acc += Lt[m * nnc + mc] * (fld(c, c->F[L], L, p, mc)[x] - fld(c, c->Fold[L], L, p, mc)[x]);
            dc[x] = acc;
        }
        if (c->p.interp_order == 4 && nc >= 3) or_prolong4_add(dim, nc, dc, ff);
        else or_prolong_add(dim, nc, dc, ff);
    }
    free(dc);
}

void or_interpolate(or_pfasst *c, int p) { or_interpolate_level(c, 0, p); }

void or_pfasst_spread(or_pfasst *c, const double *u_block)
{
    const int P = c->p.n_slices;
    memcpy(c->ublock, u_block, c->len[0] * sizeof(double));
    for (int p = 0; p < P; ++p)
        for (int m = 0; m < c->nn[0]; ++m) {
            memcpy(fld(c, c->U[0], 0, p, m), u_block, c->len[0] * sizeof(double));
            feval(c, 0, u_block, fld(c, c->F[0], 0, p, m));
        }
    for (int l = 1; l < c->nl; ++l) inject(c->p.dim, c->n[l - 1], c->ub[l - 1], c->ub[l]);
}

/* fine_send = 1: keep every slice's fine end value as the one it sends. */
static void snapshot_ends(or_pfasst *c)
{
    if (!c->p.fine_send) return;
    const int Mf = c->nn[0] - 1;
    for (int p = 0; p < c->p.n_slices; ++p)
        memcpy(c->Esnap + (size_t)p * c->len[0], fld(c, c->U[0], 0, p, Mf), c->len[0] * sizeof(double));
}

/* Predictor (Sec. 2.4): rounds j = 0..P-1; in round j every slice p >= j
 * (for j >= 1) takes the coarse end value slice p-1 had after round j-1
 * and does one coarse sweep, so slice p sweeps p+1 times. */
void or_pfasst_predictor(or_pfasst *c)
{
    if (c->nl < 2) {
        snapshot_ends(c);
        return;
    }
    const int L = c->nl - 1;
    const int P = c->p.n_slices, Mc = c->nn[L] - 1;
    const size_t lc = c->len[L];
    for (int l = 0; l < L; ++l)
        for (int p = 0; p < P; ++p) or_fas_restrict_level(c, l, p);
    double *E = (double *)malloc((size_t)P * lc * sizeof(double));
    for (int j = 0; j < P; ++j) {
        for (int p = 0; p < P; ++p) memcpy(E + p * lc, fld(c, c->U[L], L, p, Mc), lc * sizeof(double));
        for (int p = j; p < P; ++p) {
            if (j >= 1 && p >= 1) {
                double *u0 = fld(c, c->U[L], L, p, 0);
                memcpy(u0, E + (size_t)(p - 1) * lc, lc * sizeof(double));
                feval(c, L, u0, fld(c, c->F[L], L, p, 0));
            }
            or_sdc_sweep(c, L, p);
        }
    }
    free(E);
    for (int l = L - 1; l >= 0; --l)
        for (int p = 0; p < P; ++p) or_interpolate_level(c, l, p);
    snapshot_ends(c);
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
    /* the value each slice sends: its end value now (after the previous
     * iteration), or the one kept right after its last fine sweep */
    double *E = (double *)malloc((size_t)P * lf * sizeof(double));
    for (int p = 0; p < P; ++p)
        memcpy(E + p * lf, c->p.fine_send ? c->Esnap + (size_t)p * lf : fld(c, c->U[0], 0, p, Mf),
               lf * sizeof(double));
    for (int p = 1; p < P; ++p) {
        double *u0 = fld(c, c->U[0], 0, p, 0);
        memcpy(u0, E + (size_t)(p - 1) * lf, lf * sizeof(double));
        feval(c, 0, u0, fld(c, c->F[0], 0, p, 0));
    }
    free(E);
    for (int p = 0; p < P; ++p) or_sdc_sweep(c, 0, p);
    snapshot_ends(c);
    if (c->nl > 1) {
        const int L = c->nl - 1, Mc = c->nn[L] - 1;
        const size_t lc = c->len[L];
        for (int l = 0; l < L; ++l) {
            for (int p = 0; p < P; ++p) or_fas_restrict_level(c, l, p);
            /* middle levels sweep on the way down */
            if (l + 1 < L)
                for (int p = 0; p < P; ++p) or_sdc_sweep(c, l + 1, p);
        }
        for (int p = 0; p < P; ++p) {
            double *u0 = fld(c, c->U[L], L, p, 0);
            memcpy(u0, p == 0 ? c->ub[L] : fld(c, c->U[L], L, p - 1, Mc), lc * sizeof(double));
            feval(c, L, u0, fld(c, c->F[L], L, p, 0));
            or_sdc_sweep(c, L, p);
        }
        for (int l = L - 1; l >= 0; --l) {
            for (int p = 0; p < P; ++p) or_interpolate_level(c, l, p);
            /* and on the way up */
            if (l > 0)
                for (int p = 0; p < P; ++p) or_sdc_sweep(c, l, p);
        }
    }
    return or_pfasst_residual(c, NULL);
}
