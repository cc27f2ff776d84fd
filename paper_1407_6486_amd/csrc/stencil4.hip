// Fourth-order spatial discretisation on the fine level (the paper's
// fourth-order runs, Sec. 4.3) and fourth-order spatial interpolation of
// the PFASST coarse correction.
//
//  apply_L4     F = c L4 u: per axis (-u_{i-2} + 16 u_{i-1} - 30 u_i
//               + 16 u_{i+1} - u_{i+2}) / (12 h^2).  The halo holds the
//               zero boundary value one step out; two steps out the value
//               is the odd reflection -u_{1} (or -u_{n}), which keeps the
//               sine modes eigenvectors.  The field layout shares halo
//               words between rows, so that value is selected by index,
//               never read.
//  resid4       r = b - (u - alpha L4 u).
//  smooth4      one pass of weighted Jacobi (every point) or of one colour
//               of the red-black JOR: points of the colour are updated from
//               the input field (the stencil reaches same-colour points two
//               steps away), the others copied; out of place.
//  prolong4_add u += P4 e_c: tensor-product cubic Lagrange interpolation
//               (prolong4_add2: two corrections into two fields at once).
//               A fine point on a coarse point takes its value; between
//               coarse points J and J+1 the cubic through J-1 .. J+2,
//               shifted inwards next to the boundary (whose zero value is
//               one of the four points).
//
// Point-per-thread launches (tile.h); these grids are the small fine grids
// of the fourth-order configurations, not the streaming hot loop.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace pfmg {
namespace {

// 12 x (sum over axes of the 5-point fourth difference) at (i, j, k),
// 1-based, element offset o.
template <int DIM>
__device__ inline double d4sum(const double *__restrict__ u, int n, int i, int j, int k, long o, long sy, long sz)
{
    const double c = u[o];
    auto axis = [&](int x, long st) {
        // the address is clamped to the point itself where the value two
        // steps out is the reflection, so every load stays in the field
        const double m2v = u[x >= 2 ? o - 2 * st : o];
        const double p2v = u[x <= n - 1 ? o + 2 * st : o];
        const double m2 = x >= 2 ? m2v : -c;
        const double p2 = x <= n - 1 ? p2v : -c;
        return -m2 + 16.0 * u[o - st] - 30.0 * c + 16.0 * u[o + st] - p2;
    };
    double s = axis(i, 1);
    if (DIM == 3) {
        s += axis(j, sy);
        s += axis(k, sz);
    }
    return s;
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void apply_L4_kernel(Tiling t, double c, View<double> u, View<double> F)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const double ih2 = (double)(q.n + 1) * (double)(q.n + 1);
    const double d = d4sum<DIM>(fp(u, q), q.n, i, j, k, o, row_stride(q.n), plane_stride(q.n));
    fp(F, q)[o] = q.par(c) * (ih2 * (d / 12.0));
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void resid4_kernel(Tiling t, double alpha, View<double> b, View<double> u,
                                                       View<double> r)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const double ah = q.par(alpha) * (double)(q.n + 1) * (double)(q.n + 1);
    const double *uu = fp(u, q);
    const double d = d4sum<DIM>(uu, q.n, i, j, k, o, row_stride(q.n), plane_stride(q.n));
    fp(r, q)[o] = fp(b, q)[o] - (uu[o] - ah * (d / 12.0));
}

// colour < 0: every point (weighted Jacobi); 0 red, 1 black (red: 1-based
// index sum even).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void smooth4_kernel(Tiling t, double alpha, double omega, int colour,
                                                        View<double> b, View<double> src, View<double> dst)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const double *uu = fp(src, q);
    const double uc = uu[o];
    const int sum1 = DIM == 3 ? i + j + k : i;
    double v = uc;
    if (colour < 0 || (sum1 & 1) == colour) {
        const double a = q.par(alpha);
        const double ah = a * (double)(q.n + 1) * (double)(q.n + 1);
        const double diag = 1.0 + 2.5 * DIM * a * (double)(q.n + 1) * (double)(q.n + 1);
        const double d = d4sum<DIM>(uu, q.n, i, j, k, o, row_stride(q.n), plane_stride(q.n));
        const double r = fp(b, q)[o] - (uc - ah * (d / 12.0));
        v = uc + omega * r / diag;
    }
    fp(dst, q)[o] = v;
}

// Cubic Lagrange weights of fine 1-based index x on coarse 1-based
// indices idx (0 and nc+1 are the boundary).  Returns the count (1 or 4).
// A fine point between coarse points sits at their midpoint, so the
// weights are constants: (-1, 9, 9, -1)/16 on J-1 .. J+2, and next to a
// boundary the shifted stencils (5, 15, -5, 1)/16 and (1, -5, 15, 5)/16
// (exact dyadic values of the Lagrange basis at the midpoint).
__device__ inline int cubic_w(int x, int nc, int *idx, double *w)
{
    if ((x & 1) == 0) {
        idx[0] = x / 2;
        w[0] = 1.0;
        return 1;
    }
    const int J = (x - 1) / 2;
    int lo;
    if (J == 0) {
        lo = 0;
        w[0] = 5.0 / 16; w[1] = 15.0 / 16; w[2] = -5.0 / 16; w[3] = 1.0 / 16;
    } else if (J == nc) {
        lo = nc - 2;
        w[0] = 1.0 / 16; w[1] = -5.0 / 16; w[2] = 15.0 / 16; w[3] = 5.0 / 16;
    } else {
        lo = J - 1;
        w[0] = -1.0 / 16; w[1] = 9.0 / 16; w[2] = 9.0 / 16; w[3] = -1.0 / 16;
    }
    for (int a = 0; a < 4; ++a) idx[a] = lo + a;
    return 4;
}

// Launched on the fine grids; ec on the coarse grids nc = (n+1)/2 - 1.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void prolong4_add_kernel(Tiling t, View<double> ec, View<double> u)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const int nc = coarser(q.n);
    const long syc = row_stride(nc), szc = plane_stride(nc);
    const double *e = fp(ec, q);
    int ix[4], iy[4] = {0, 0, 0, 0}, iz[4] = {0, 0, 0, 0};
    double wx[4], wy[4] = {1.0, 0, 0, 0}, wz[4] = {1.0, 0, 0, 0};
    const int cx = cubic_w(i, nc, ix, wx);
    const int cy = DIM == 3 ? cubic_w(j, nc, iy, wy) : 1;
    const int cz = DIM == 3 ? cubic_w(k, nc, iz, wz) : 1;
    double acc = 0.0;
    for (int c = 0; c < cz; ++c)
        for (int b = 0; b < cy; ++b)
            for (int a = 0; a < cx; ++a) {
                const long oc = DIM == 3 ? (long)ix[a] + (long)iy[b] * syc + (long)iz[c] * szc : (long)ix[a];
                acc += wz[c] * wy[b] * wx[a] * e[oc];
            }
    fp(u, q)[o] += acc;
}

// prolong4_add of two corrections at once (U's and F's in PFASST
// interpolation): the same indices and weights, each sum accumulated as in
// prolong4_add_kernel.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void prolong4_add2_kernel(Tiling t, View<double> ec, View<double> u,
                                                              View<double> ec2, View<double> u2)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const int nc = coarser(q.n);
    const long syc = row_stride(nc), szc = plane_stride(nc);
    const double *e = fp(ec, q), *e2 = fp(ec2, q);
    int ix[4], iy[4] = {0, 0, 0, 0}, iz[4] = {0, 0, 0, 0};
    double wx[4], wy[4] = {1.0, 0, 0, 0}, wz[4] = {1.0, 0, 0, 0};
    const int cx = cubic_w(i, nc, ix, wx);
    const int cy = DIM == 3 ? cubic_w(j, nc, iy, wy) : 1;
    const int cz = DIM == 3 ? cubic_w(k, nc, iz, wz) : 1;
    double acc = 0.0, acc2 = 0.0;
    for (int c = 0; c < cz; ++c)
        for (int b = 0; b < cy; ++b)
            for (int a = 0; a < cx; ++a) {
                const long oc = DIM == 3 ? (long)ix[a] + (long)iy[b] * syc + (long)iz[c] * szc : (long)ix[a];
                const double w = wz[c] * wy[b] * wx[a];
                acc += w * e[oc];
                acc2 += w * e2[oc];
            }
    fp(u, q)[o] += acc;
    fp(u2, q)[o] += acc2;
}

inline dim3 grid4(const Tiling &t) { return dim3((unsigned)grid_blocks(t)); }

#define PFMG_DISPATCH4(t, KER, ...)                                                         \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3><<<grid4(t), BLOCK, 0, s>>>(__VA_ARGS__);                   \
        else KER<1><<<grid4(t), BLOCK, 0, s>>>(__VA_ARGS__);                                \
        return hipGetLastError();                                                           \
    } while (0)

}  // namespace

namespace k {

hipError_t apply_L4(const Tiling &t, double nu, View<double> u, View<double> F, hipStream_t s)
{
    PFMG_DISPATCH4(t, apply_L4_kernel, t, nu, u, F);
}

hipError_t resid4(const Tiling &t, double alpha, View<double> b, View<double> u, View<double> r, hipStream_t s)
{
    PFMG_DISPATCH4(t, resid4_kernel, t, alpha, b, u, r);
}

hipError_t smooth4(const Tiling &t, double alpha, double omega, int colour, View<double> b, View<double> src,
                   View<double> dst, hipStream_t s)
{
    if (colour > 1) return hipErrorInvalidValue;
    PFMG_DISPATCH4(t, smooth4_kernel, t, alpha, omega, colour, b, src, dst);
}

hipError_t prolong4_add(const Tiling &t, View<double> ec, View<double> u, hipStream_t s)
{
    for (int sg = 0; sg < t.nseg; ++sg)
        if (t.seg_count(sg) > 0 && coarser(t.seg_n(sg)) < 3) return hipErrorInvalidValue;
    PFMG_DISPATCH4(t, prolong4_add_kernel, t, ec, u);
}

hipError_t prolong4_add2(const Tiling &t, View<double> ec, View<double> u, View<double> ec2, View<double> u2,
                         hipStream_t s)
{
    for (int sg = 0; sg < t.nseg; ++sg)
        if (t.seg_count(sg) > 0 && coarser(t.seg_n(sg)) < 3) return hipErrorInvalidValue;
    PFMG_DISPATCH4(t, prolong4_add2_kernel, t, ec, u, ec2, u2);
}

}  // namespace k
}  // namespace pfmg
