/*
 * Collocation matrices for the oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Quadrature nodes and the integration matrix of Sec. 2.1 (the q_{m,i}
 * with int_{t0}^{tm} g ~ dt sum_i q_{m,i} g(t_i)), the node-to-node
 * differences used in eq. sdc-be, and the backward-Euler substeps of
 * eq. Qbe.  Two node families: Gauss-Lobatto, whose first row of Q is
 * zero (node 0 is the left end point) but q_{m,0} != 0 for m >= 1; and the
 * uniform nodes of the paper's second- and fourth-order methods (Sec. 3),
 * whose quadrature leaves out the left end point: f is interpolated
 * through nodes 1..M only, so the whole column q_{.,0} is zero.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

typedef long double ld;

/* Legendre P_M(x) and P_{M-1}(x) by the three-term recurrence. */
static void legendre(int M, ld x, ld *pm, ld *pm1)
{
    ld p0 = 1.0L, p1 = x;
    if (M == 0) { *pm = 1.0L; *pm1 = 0.0L; return; }
    for (int k = 1; k < M; ++k) {
        ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
    }
    *pm = p1;
    *pm1 = p0;
}

static int lobatto_ld(int nnodes, ld *s)
{
    if (nnodes < 2 || nnodes > 16) return -1;
    int M = nnodes - 1;
    s[0] = 0.0L;
    s[M] = 1.0L;
    /* Interior nodes: roots of P'_M on (-1,1), mapped to (0,1).  Newton
     * from the Chebyshev-Lobatto points; P'' from Legendre's equation. */
    for (int j = 1; j < M; ++j) {
        ld x = -cosl(3.14159265358979323846264338327950288L * j / M);
        for (int it = 0; it < 100; ++it) {
            ld p, pm1;
            legendre(M, x, &p, &pm1);
            ld dp = M * (x * p - pm1) / (x * x - 1.0L);
            ld d2p = (2.0L * x * dp - M * (M + 1) * p) / (1.0L - x * x);
            ld dx = dp / d2p;
            x -= dx;
            if (fabsl(dx) < 1e-30L) break;
        }
        s[j] = (x + 1.0L) / 2.0L;
    }
    return 0;
}

int or_lobatto_nodes(int nnodes, double *s)
{
    ld t[16];
    if (lobatto_ld(nnodes, t)) return -1;
    for (int i = 0; i < nnodes; ++i) s[i] = (double)t[i];
    return 0;
}

/* Monomial coefficients c[0..M] of the Lagrange basis polynomial l_i. */
static void lagrange_coeffs(int nn, const ld *s, int i, ld *c)
{
    ld denom = 1.0L;
    for (int k = 0; k < nn; ++k) c[k] = 0.0L;
    c[0] = 1.0L;
    int deg = 0;
    for (int j = 0; j < nn; ++j) {
        if (j == i) continue;
        /* multiply by (x - s_j) */
        for (int k = deg + 1; k >= 1; --k) c[k] = c[k - 1] - s[j] * c[k];
        c[0] = -s[j] * c[0];
        ++deg;
        denom *= (s[i] - s[j]);
    }
    for (int k = 0; k < nn; ++k) c[k] /= denom;
}

int or_uniform_nodes(int nnodes, double *s)
{
    if (nnodes < 2 || nnodes > 16) return -1;
    for (int i = 0; i < nnodes; ++i) s[i] = (double)i / (double)(nnodes - 1);
    return 0;
}

/* Uniform nodes without the left end point: Lagrange basis of the M nodes
 * s_1..s_M (a polynomial of degree M-1 through f_1..f_M), integrated from
 * 0 to every s_m.  Node values are m/M formed in long double. */
static int qmat_uniform(int nnodes, double *Q, double *S, double *d)
{
    const int M = nnodes - 1;
    ld s[16], Ql[16 * 16], c[17];
    for (int i = 0; i <= M; ++i) s[i] = (ld)i / (ld)M;
    for (int q = 0; q < nnodes * nnodes; ++q) Ql[q] = 0.0L;
    for (int i = 1; i <= M; ++i) {
        /* basis polynomial of node i over the nodes 1..M */
        lagrange_coeffs(M, s + 1, i - 1, c);
        for (int m = 0; m <= M; ++m) {
            ld acc = 0.0L, pw = s[m];
            for (int k = 0; k < M; ++k) {
                acc += c[k] * pw / (k + 1);
                pw *= s[m];
            }
            Ql[m * nnodes + i] = acc;
        }
    }
    for (int q = 0; q < nnodes * nnodes; ++q) Q[q] = (double)Ql[q];
    if (S)
        for (int m = 0; m < M; ++m)
            for (int i = 0; i < nnodes; ++i)
                S[m * nnodes + i] = (double)(Ql[(m + 1) * nnodes + i] - Ql[m * nnodes + i]);
    if (d) {
        d[0] = 0.0;
        for (int m = 1; m <= M; ++m) d[m] = (double)(s[m] - s[m - 1]);
    }
    return 0;
}

int or_qmat_family(int nnodes, const double *s, int family, double *Q, double *S, double *d)
{
    if (nnodes < 2 || nnodes > 16) return -1;
    if (family == OR_NODES_UNIFORM) return qmat_uniform(nnodes, Q, S, d);
    if (family != OR_NODES_LOBATTO) return -1;
    return or_qmat(nnodes, s, Q, S, d);
}

int or_qmat(int nnodes, const double *s_in, double *Q, double *S, double *d)
{
    if (nnodes < 2 || nnodes > 16) return -1;
    ld s[16], Ql[16 * 16], c[17];
    /* Nodes are recomputed in long double when they are the Lobatto set;
     * the double inputs are used otherwise. */
    ld lob[16];
    int is_lob = (lobatto_ld(nnodes, lob) == 0);
    for (int i = 0; i < nnodes; ++i) {
        if (is_lob && (double)lob[i] == s_in[i]) s[i] = lob[i];
        else s[i] = (ld)s_in[i];
    }
    for (int i = 0; i < nnodes; ++i) {
        lagrange_coeffs(nnodes, s, i, c);
        for (int m = 0; m < nnodes; ++m) {
            /* int_0^{s_m} l_i = sum_k c_k s_m^{k+1}/(k+1) */
            ld acc = 0.0L, pw = s[m];
            for (int k = 0; k < nnodes; ++k) {
                acc += c[k] * pw / (k + 1);
                pw *= s[m];
            }
            Ql[m * nnodes + i] = acc;
        }
    }
    for (int m = 0; m < nnodes; ++m)
        for (int i = 0; i < nnodes; ++i) Q[m * nnodes + i] = (double)Ql[m * nnodes + i];
    if (S)
        for (int m = 0; m + 1 < nnodes; ++m)
            for (int i = 0; i < nnodes; ++i)
                S[m * nnodes + i] = (double)(Ql[(m + 1) * nnodes + i] - Ql[m * nnodes + i]);
    if (d) {
        d[0] = 0.0;
        for (int m = 1; m < nnodes; ++m) d[m] = (double)(s[m] - s[m - 1]);
    }
    return 0;
}

int or_interp_matrix(int nfn, const double *sf, int ncn, const double *sc,
                     double *L)
{
    if (ncn < 1 || ncn > 16) return -1;
    for (int mf = 0; mf < nfn; ++mf) {
        for (int mc = 0; mc < ncn; ++mc) {
            ld v = 1.0L;
            for (int j = 0; j < ncn; ++j) {
                if (j == mc) continue;
                v *= ((ld)sf[mf] - (ld)sc[j]) / ((ld)sc[mc] - (ld)sc[j]);
            }
            L[mf * ncn + mc] = (double)v;
        }
    }
    return 0;
}
