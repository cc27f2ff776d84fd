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
