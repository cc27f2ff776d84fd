/*
 * Stencils, multigrid and the node-solve policy for the oracle
 * (TEST INFRASTRUCTURE ONLY).
 *
 * Spatial operator: the second-order finite-difference Laplacian with
 * homogeneous Dirichlet data (Sec. 4.1 for 1D, Sec. 4.2 for the 3D
 * 7-point form).  Implicit node solve: (I - alpha L_h) u = b, the linear
 * SDC substep of eq. SDCcompactLIII with alpha = nu * dt_m.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define REAL double
#define SFX or
#include "mg_impl.h"
#undef REAL
#undef SFX

#define REAL float
#define SFX orf
#include "mg_impl.h"
#undef REAL
#undef SFX

void or_lap(int dim, int n, const double *u, double *out)
{
    const double ih2 = (double)(n + 1) * (double)(n + 1);   /* 1/h^2, exact */
    const int ny = dim >= 2 ? n : 1, nz = dim >= 3 ? n : 1;
#pragma omp parallel for schedule(static) if (nz > 8)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < n; ++i) {
                size_t x = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
                out[x] = ih2 * or_d2(dim, n, u, i, j, k);
            }
}

void or_helm(int dim, int n, double alpha, const double *u, double *out)
{
    const double ah = alpha * (double)(n + 1) * (double)(n + 1);
    const int ny = dim >= 2 ? n : 1, nz = dim >= 3 ? n : 1;
#pragma omp parallel for schedule(static) if (nz > 8)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < n; ++i) {
                size_t x = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
                out[x] = u[x] - ah * or_d2(dim, n, u, i, j, k);
            }
}

double or_norm_inf(size_t len, const double *v)
{
    double m = 0.0;
    for (size_t x = 0; x < len; ++x) {
        double a = fabs(v[x]);
        if (a > m || a != a) m = a;      /* NaN propagates */
        if (m != m) return m;
    }
    return m;
}

/* One step of the mixed-precision form: FP64 residual, FP32 V-cycle from a
 * zero correction, FP64 update. */
static void ir_step(int dim, int n, double alpha, const or_mg_policy *pol,
                    const double *b, double *u)
{
    const size_t len = or_len(dim, n);
    double *r = (double *)malloc(len * sizeof(double));
    float *r32 = (float *)malloc(len * sizeof(float));
    float *e32 = (float *)calloc(len, sizeof(float));
    or_resid(dim, n, alpha, b, u, r);
    for (size_t x = 0; x < len; ++x) r32[x] = (float)r[x];
    orf_vcycle(dim, n, alpha, pol->smoother, pol->omega, pol->nu1, pol->nu2, r32, e32);
    for (size_t x = 0; x < len; ++x) u[x] = u[x] + (double)e32[x];
    free(r);
    free(r32);
    free(e32);
}

static double resid_norm(int dim, int n, double alpha, const double *b, const double *u)
{
    const size_t len = or_len(dim, n);
    double *r = (double *)malloc(len * sizeof(double));
    or_resid(dim, n, alpha, b, u, r);
    double v = or_norm_inf(len, r);
    free(r);
    return v;
}

/* Fixed number of cycles (the inexact solves of ISDC, Sec. 2.3.1), or the
 * full solve of Sec. 4.2.1: repeat while |r| > tol |b| and each cycle cuts
 * the residual below stall * the previous one, at most max_cycles. */
int or_mg_solve(int dim, int n, double alpha, const or_mg_policy *pol,
                const double *b, double *u, double *relres)
{
    const size_t len = or_len(dim, n);
    int done = 0;
    if (pol->cycles > 0) {
        for (int c = 0; c < pol->cycles; ++c) {
            if (pol->mixed) ir_step(dim, n, alpha, pol, b, u);
            else or_vcycle(dim, n, alpha, pol->smoother, pol->omega, pol->nu1, pol->nu2, b, u);
        }
        done = pol->cycles;
        if (relres) {
            double nb = or_norm_inf(len, b);
            double nr = resid_norm(dim, n, alpha, b, u);
            *relres = nb > 0 ? nr / nb : nr;
        }
        return done;
    }
    double nb = or_norm_inf(len, b);
    double r = resid_norm(dim, n, alpha, b, u);
    while (done < pol->max_cycles && r > pol->tol * nb) {
        if (pol->mixed) ir_step(dim, n, alpha, pol, b, u);
        else or_vcycle(dim, n, alpha, pol->smoother, pol->omega, pol->nu1, pol->nu2, b, u);
        ++done;
        double rn = resid_norm(dim, n, alpha, b, u);
        int stalled = !(rn < pol->stall * r);
        r = rn;
        if (stalled) break;
    }
    if (relres) *relres = nb > 0 ? r / nb : r;
    return done;
}

/* ------------------------------------------------------------------
 * Fourth-order spatial discretisation (the paper's fourth-order runs,
 * Sec. 4.3): per dimension (-u_{i-2} + 16 u_{i-1} - 30 u_i + 16 u_{i+1}
 * - u_{i+2}) / (12 h^2).  Next to the boundary the value two points out
 * lies outside the domain; it is the odd reflection of the interior value
 * (u(-h) = -u(h)), consistent with the zero Dirichlet data, so that the
 * sine modes stay eigenvectors.
 * ------------------------------------------------------------------ */

/* u along one axis at offset o from 0-based index x (|o| <= 2): zero on
 * the boundary, the reflected interior value one step beyond it. */
static inline double ax4(const double *u, int n, int i, int j, int k, int axis, int o)
{
    int c[3] = {i, j, k};
    int x = c[axis] + o;
    double sgn = 1.0;
    if (x == -1 || x == n) return 0.0;
    if (x == -2) { x = 0; sgn = -1.0; }
    if (x == n + 1) { x = n - 1; sgn = -1.0; }
    c[axis] = x;
    return sgn * u[(size_t)c[0] + (size_t)n * ((size_t)c[1] + (size_t)n * (size_t)c[2])];
}

/* sum over dimensions of the 5-point fourth difference times 12 (not yet
 * divided by 12 h^2) */
static inline double d4(int dim, int n, const double *u, int i, int j, int k)
{
    double s = 0.0;
    for (int a = 0; a < dim; ++a)
        s += (-ax4(u, n, i, j, k, a, -2) + 16.0 * ax4(u, n, i, j, k, a, -1) - 30.0 * ax4(u, n, i, j, k, a, 0)
              + 16.0 * ax4(u, n, i, j, k, a, 1) - ax4(u, n, i, j, k, a, 2));
    return s;
}

void or_lap4(int dim, int n, const double *u, double *out)
{
    const double ih2 = (double)(n + 1) * (double)(n + 1);
    const int ny = dim >= 2 ? n : 1, nz = dim >= 3 ? n : 1;
#pragma omp parallel for schedule(static) if (nz > 8)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < n; ++i)
                out[(size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k)] = ih2 * (d4(dim, n, u, i, j, k) / 12.0);
}

void or_resid4(int dim, int n, double alpha, const double *b, const double *u, double *r)
{
    const double ah = alpha * (double)(n + 1) * (double)(n + 1);
    const int ny = dim >= 2 ? n : 1, nz = dim >= 3 ? n : 1;
#pragma omp parallel for schedule(static) if (nz > 8)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < n; ++i) {
                const size_t x = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
                r[x] = b[x] - (u[x] - ah * (d4(dim, n, u, i, j, k) / 12.0));
            }
}

/* Smoothing for (I - alpha L4): weighted Jacobi on every point, or the
 * red-black JOR of Sec. 4.3: the points of one colour updated together from
 * the values before that colour's pass (the stencil reaches same-colour
 * points two steps away), red then black.  diag(I - alpha L4) =
 * 1 + 30 dim alpha / (12 h^2). */
void or_smooth4(int dim, int n, double alpha, int smoother, double omega, const double *b, double *u)
{
    const size_t len = or_len(dim, n);
    const double diag = 1.0 + 2.5 * dim * alpha * (double)(n + 1) * (double)(n + 1);
    const int ny = dim >= 2 ? n : 1, nz = dim >= 3 ? n : 1;
    double *r = (double *)malloc(len * sizeof(double));
    for (int colour = 0; colour < (smoother == OR_JACOBI ? 1 : 2); ++colour) {
        or_resid4(dim, n, alpha, b, u, r);
#pragma omp parallel for schedule(static) if (nz > 8)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < n; ++i) {
                    const int sum1 = (i + 1) + (dim >= 2 ? j + 1 : 0) + (dim >= 3 ? k + 1 : 0);
                    if (smoother != OR_JACOBI && (sum1 & 1) != colour) continue;
                    const size_t x = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
                    u[x] = u[x] + omega * r[x] / diag;
                }
    }
    free(r);
}

/* V-cycle for (I - alpha L4): the finest level smooths and forms its
 * residual with L4; the correction equation below it is the second-order
 * (I - alpha L_2h), solved by the second-order V-cycle. */
void or_vcycle4(int dim, int n, double alpha, int smoother, double omega, int nu1, int nu2,
                const double *b, double *u)
{
    if (n <= 2) {
        /* no coarser grid: smoothing on L4 only (not reached by the
         * library's grids, n >= 3 odd) */
        for (int s = 0; s < nu1 + nu2; ++s) or_smooth4(dim, n, alpha, smoother, omega, b, u);
        return;
    }
    const size_t len = or_len(dim, n);
    const int nc = (n + 1) / 2 - 1;
    const size_t lenc = or_len(dim, nc);
    for (int s = 0; s < nu1; ++s) or_smooth4(dim, n, alpha, smoother, omega, b, u);
    double *r = (double *)malloc(len * sizeof(double));
    double *bc = (double *)malloc(lenc * sizeof(double));
    double *ec = (double *)calloc(lenc, sizeof(double));
    or_resid4(dim, n, alpha, b, u, r);
    or_restrict_fw(dim, n, r, bc);
    or_vcycle(dim, nc, alpha, smoother, omega, nu1, nu2, bc, ec);
    or_prolong_add(dim, nc, ec, u);
    free(r);
    free(bc);
    free(ec);
    for (int s = 0; s < nu2; ++s) or_smooth4(dim, n, alpha, smoother, omega, b, u);
}

static double resid4_norm(int dim, int n, double alpha, const double *b, const double *u)
{
    const size_t len = or_len(dim, n);
    double *r = (double *)malloc(len * sizeof(double));
    or_resid4(dim, n, alpha, b, u, r);
    double v = or_norm_inf(len, r);
    free(r);
    return v;
}

/* or_mg_solve for (I - alpha L4) (no mixed-precision form). */
int or_mg_solve4(int dim, int n, double alpha, const or_mg_policy *pol, const double *b, double *u, double *relres)
{
    const size_t len = or_len(dim, n);
    int done = 0;
    const double nb = or_norm_inf(len, b);
    if (pol->cycles > 0) {
        for (int c = 0; c < pol->cycles; ++c)
            or_vcycle4(dim, n, alpha, pol->smoother, pol->omega, pol->nu1, pol->nu2, b, u);
        if (relres) {
            const double nr = resid4_norm(dim, n, alpha, b, u);
            *relres = nb > 0 ? nr / nb : nr;
        }
        return pol->cycles;
    }
    double r = resid4_norm(dim, n, alpha, b, u);
    while (done < pol->max_cycles && r > pol->tol * nb) {
        or_vcycle4(dim, n, alpha, pol->smoother, pol->omega, pol->nu1, pol->nu2, b, u);
        ++done;
        const double rn = resid4_norm(dim, n, alpha, b, u);
        const int stalled = !(rn < pol->stall * r);
        r = rn;
        if (stalled) break;
    }
    if (relres) *relres = nb > 0 ? r / nb : r;
    return done;
}

/* Cubic Lagrange weights of fine 1-based index i on coarse 1-based indices;
 * coarse indices 0 and nc+1 are the zero boundary values. */
static int cubic_weights(int i, int nc, int *idx, double *w)
{
    if ((i & 1) == 0) {
        idx[0] = i / 2;
        w[0] = 1.0;
        return 1;
    }
    const int J = (i - 1) / 2;            /* between coarse J and J+1 */
    int lo = J - 1;
    if (lo < 0) lo = 0;
    if (lo + 3 > nc + 1) lo = nc + 1 - 3;
    const double x = J + 0.5;
    for (int q = 0; q < 4; ++q) {
        double v = 1.0;
        for (int r = 0; r < 4; ++r)
            if (r != q) v *= (x - (lo + r)) / (double)((lo + q) - (lo + r));
        idx[q] = lo + q;
        w[q] = v;
    }
    return 4;
}

void or_prolong4_add(int dim, int nc, const double *ec, double *u)
{
    const int n = 2 * (nc + 1) - 1;
    const int ny = dim >= 2 ? n : 1, nz = dim >= 3 ? n : 1;
#pragma omp parallel for schedule(static) if (nz > 8)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < n; ++i) {
                int ix[4], iy[4] = {1}, iz[4] = {1};
                double wx[4], wy[4] = {1.0}, wz[4] = {1.0};
                const int cx = cubic_weights(i + 1, nc, ix, wx);
                const int cy = dim >= 2 ? cubic_weights(j + 1, nc, iy, wy) : 1;
                const int cz = dim >= 3 ? cubic_weights(k + 1, nc, iz, wz) : 1;
                double acc = 0.0;
                for (int c = 0; c < cz; ++c)
                    for (int b = 0; b < cy; ++b)
                        for (int a = 0; a < cx; ++a) {
                            const double v = or_at(ec, nc, ix[a] - 1, dim >= 2 ? iy[b] - 1 : 0, dim >= 3 ? iz[c] - 1 : 0);
                            acc += wz[c] * wy[b] * wx[a] * v;
                        }
                u[(size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k)] += acc;
            }
}
