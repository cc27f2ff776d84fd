// Collocation matrices of the library (host, long double, rounded once).
//
// Gauss-Lobatto nodes on [0, 1]: the end points plus the roots of P'_M,
// bracketed by sign changes on a fine grid and polished by Newton.  Uniform
// nodes: m / M, with a quadrature that leaves out the left end point (the
// second- and fourth-order methods of Sec. 3).  The integration matrix of
// Sec. 2.1, Q[m][i] = int_0^{s_m} l_i, is obtained from exactness on
// monomials: sum_i Q[m][i] s_i^j = s_m^{j+1} / (j+1) over the quadrature's
// nodes (all of them, or 1..M) and degrees j below their count, a
// Vandermonde system solved by Gaussian elimination with partial pivoting.
// S[m][i] = Q[m+1][i] - Q[m][i] are the node-to-node integrals of eq.
// sdc-be; d[m] = s_m - s_{m-1} the backward-Euler substeps of eq. Qbe.
#include <cmath>
#include <vector>

#include "../../include/pfmg.h"
#include "collocation.h"

namespace pfmg {
namespace {

using ld = long double;

// P'_M(x) and P''_M(x) via P'_{k+1} = P'_{k-1} + (2k+1) P_k and the same
// recurrence differentiated once more.
void legendre_d(int M, ld x, ld &d1, ld &d2)
{
    std::vector<ld> P(M + 1), D(M + 1), D2(M + 1);
    P[0] = 1; D[0] = 0; D2[0] = 0;
    if (M >= 1) { P[1] = x; D[1] = 1; D2[1] = 0; }
    for (int k = 1; k < M; ++k) {
        P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
        D[k + 1] = D[k - 1] + (2 * k + 1) * P[k];
        D2[k + 1] = D2[k - 1] + (2 * k + 1) * D[k];
    }
    d1 = D[M];
    d2 = D2[M];
}

}  // namespace

bool lobatto_nodes_ld(int nnodes, long double *s)
{
    if (nnodes < 2 || nnodes > 16) return false;
    const int M = nnodes - 1;
    std::vector<ld> roots;
    const int grid = 4000;
    ld xa = -1 + 1e-12L, fa, tmp;
    legendre_d(M, xa, fa, tmp);
    for (int g = 1; g <= grid; ++g) {
        ld xb = -1 + 2.0L * g / grid;
        if (g == grid) xb = 1 - 1e-12L;
        ld fb;
        legendre_d(M, xb, fb, tmp);
        if ((fa < 0) != (fb < 0)) {
            ld lo = xa, hi = xb, flo = fa;
            for (int it = 0; it < 200 && hi - lo > 1e-30L; ++it) {
                ld mid = (lo + hi) / 2, fm;
                legendre_d(M, mid, fm, tmp);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
            }
            ld x = (lo + hi) / 2;
            for (int it = 0; it < 4; ++it) {
                ld f1, f2;
                legendre_d(M, x, f1, f2);
                if (f2 == 0) break;
                x -= f1 / f2;
            }
            roots.push_back(x);
        }
        xa = xb;
        fa = fb;
    }
    if ((int)roots.size() != M - 1) return false;
    s[0] = 0;
    for (int j = 0; j < M - 1; ++j) s[j + 1] = (roots[j] + 1) / 2;
    s[M] = 1;
    return true;
}

bool family_nodes_ld(int family, int nnodes, long double *s)
{
    if (family == PFMG_NODES_LOBATTO) return lobatto_nodes_ld(nnodes, s);
    if (family != PFMG_NODES_UNIFORM || nnodes < 2 || nnodes > 16) return false;
    for (int m = 0; m < nnodes; ++m) s[m] = (ld)m / (ld)(nnodes - 1);
    return true;
}

bool collocation_matrices(int nnodes, const long double *s, double *Q, double *S, double *d, int first)
{
    if (nnodes < 2 || nnodes > 16 || first < 0 || first > 1) return false;
    // the quadrature's nodes are s[first .. nnodes-1]: nq of them
    const int nq = nnodes - first;
    const long double *sq = s + first;
    const int nn = nq;
    std::vector<ld> Ql(nnodes * nnodes, 0.0L);
    for (int m = 0; m < nnodes; ++m) {
        // V^T x = rhs with V[i][j] = sq_i^j: rows j, columns i.
        std::vector<ld> A(nn * nn), r(nn);
        for (int j = 0; j < nn; ++j) {
            for (int i = 0; i < nn; ++i) A[j * nn + i] = std::pow(sq[i], (ld)j);
            r[j] = std::pow(s[m], (ld)(j + 1)) / (j + 1);
        }
        for (int c = 0; c < nn; ++c) {
            int piv = c;
            for (int q = c + 1; q < nn; ++q)
                if (std::fabs(A[q * nn + c]) > std::fabs(A[piv * nn + c])) piv = q;
            if (A[piv * nn + c] == 0) return false;
            if (piv != c) {
                for (int q = 0; q < nn; ++q) std::swap(A[c * nn + q], A[piv * nn + q]);
                std::swap(r[c], r[piv]);
            }
            for (int q = c + 1; q < nn; ++q) {
                ld f = A[q * nn + c] / A[c * nn + c];
                for (int w = c; w < nn; ++w) A[q * nn + w] -= f * A[c * nn + w];
                r[q] -= f * r[c];
            }
        }
        for (int c = nn - 1; c >= 0; --c) {
            ld acc = r[c];
            for (int w = c + 1; w < nn; ++w) acc -= A[c * nn + w] * r[w];
            r[c] = acc / A[c * nn + c];
        }
        for (int i = 0; i < nn; ++i) Ql[m * nnodes + first + i] = (m == 0) ? 0.0L : r[i];
    }
    for (int q = 0; q < nnodes * nnodes; ++q) Q[q] = (double)Ql[q];
    for (int m = 0; m + 1 < nnodes; ++m)
        for (int i = 0; i < nnodes; ++i) S[m * nnodes + i] = (double)(Ql[(m + 1) * nnodes + i] - Ql[m * nnodes + i]);
    d[0] = 0;
    for (int m = 1; m < nnodes; ++m) d[m] = (double)(s[m] - s[m - 1]);
    return true;
}

void lagrange_interp(int nf, const long double *sf, int nc, const long double *sc, double *L)
{
    for (int mf = 0; mf < nf; ++mf)
        for (int mc = 0; mc < nc; ++mc) {
            ld v = 1;
            for (int q = 0; q < nc; ++q)
                if (q != mc) v *= (sf[mf] - sc[q]) / (sc[mc] - sc[q]);
            L[mf * nc + mc] = (double)v;
        }
}

}  // namespace pfmg
