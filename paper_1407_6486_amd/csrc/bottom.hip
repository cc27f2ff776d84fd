// The lower part of a V-cycle in one launch: one workgroup per field solves
// (I - alpha L_h) u = b with a V(nu1, nu2) cycle from grid n0 down to the
// exact solve, entirely in LDS.
//
// Used for the grids below the streaming kernels' efficient range (3D:
// n <= 15, 1D: every grid), where the per-level launches of the big-grid
// path would cost more than the work.  The steps are those of the V-cycle
// of Sec. 4.1.1 / 4.2.1: smoothing (weighted Jacobi or red-black), residual
// with full-weighting restriction, recursive correction from zero,
// d-linear prolongation, smoothing; exact solve on n in {1, 2}.  Grids are
// stored densely in LDS (no halo); neighbours outside the grid are the zero
// Dirichlet data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "../../include/pfmg.h"
#include "kernels.h"

namespace pfmg {
namespace {

constexpr int MAXL = 16;
constexpr int BT = 1024;          // 3D: 16 x 16 x 4 threads; 1D: 1024 x 1 x 1

// Visit every point of an n^DIM grid: coordinates come from the thread
// index (no integer division), p is the dense index.
template <int DIM, class F>
__device__ inline void for_points(int n, F f)
{
    if (DIM == 3) {
        for (int k = threadIdx.z; k < n; k += blockDim.z)
            for (int j = threadIdx.y; j < n; j += blockDim.y)
                for (int i = threadIdx.x; i < n; i += blockDim.x) f(i + n * (j + n * k), i, j, k);
    } else {
        for (int i = threadIdx.x; i < n; i += blockDim.x) f(i, i, 0, 0);
    }
}

__host__ __device__ inline int ipow(int n, int dim) { return dim == 3 ? n * n * n : n; }

template <int DIM, typename T>
struct Grid {
    T *u, *b, *t;
    int n;
    __device__ T at(const T *a, int i, int j, int k) const
    {
        if (i < 0 || i >= n) return (T)0;
        if (DIM == 3 && (j < 0 || j >= n || k < 0 || k >= n)) return (T)0;
        return a[DIM == 3 ? i + n * (j + n * k) : i];
    }
    __device__ void coords(int p, int &i, int &j, int &k) const
    {
        if (DIM == 3) { i = p % n; j = (p / n) % n; k = p / (n * n); }
        else { i = p; j = k = 0; }
    }
    __device__ T d2(const T *a, int i, int j, int k) const
    {
        const T c = a[DIM == 3 ? i + n * (j + n * k) : i];
        T s = at(a, i - 1, j, k) + at(a, i + 1, j, k);
        if (DIM == 3) s += (at(a, i, j - 1, k) + at(a, i, j + 1, k)) + (at(a, i, j, k - 1) + at(a, i, j, k + 1));
        return s - (T)(2 * DIM) * c;
    }
};

template <int DIM, typename T>
__device__ void smooth(Grid<DIM, T> &g, T ah, T winv, int smoother, int sweeps, bool from_zero)
{
    if (sweeps == 0 && from_zero) {
        for_points<DIM>(g.n, [&](int p, int, int, int) { g.u[p] = (T)0; });
        __syncthreads();
        return;
    }
    for (int s = 0; s < sweeps; ++s) {
        const bool z = s == 0 && from_zero;
        if (smoother == PFMG_SMOOTH_RBGS) {
            for (int colour = 0; colour < 2; ++colour) {
                for_points<DIM>(g.n, [&](int p, int i, int j, int k) {
                    const int par = (DIM == 3 ? (i + j + k + 3) : (i + 1)) & 1;   // 1-based parity
                    if (z && colour == 0) {
                        g.u[p] = par == 0 ? winv * g.b[p] : (T)0;
                        return;
                    }
                    if (par != colour) return;
                    const T uc = g.u[p];
                    g.u[p] = uc + winv * (g.b[p] - (uc - ah * g.d2(g.u, i, j, k)));
                });
                __syncthreads();
            }
        } else {
            for_points<DIM>(g.n, [&](int p, int i, int j, int k) {
                if (z) {
                    g.t[p] = winv * g.b[p];
                } else {
                    const T uc = g.u[p];
                    g.t[p] = uc + winv * (g.b[p] - (uc - ah * g.d2(g.u, i, j, k)));
                }
            });
            __syncthreads();
            for_points<DIM>(g.n, [&](int p, int, int, int) { g.u[p] = g.t[p]; });
            __syncthreads();
        }
    }
}

template <int DIM, typename T>
__device__ void resid_restrict(const Grid<DIM, T> &f, Grid<DIM, T> &c, T ah)
{
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    for_points<DIM>(c.n, [&](int p, int I, int J, int K) {
        const int fi = 2 * I + 1, fj = DIM == 3 ? 2 * J + 1 : 0, fk = DIM == 3 ? 2 * K + 1 : 0;
        T acc = 0;
#pragma unroll 1
        for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
#pragma unroll 1
            for (int oy = (DIM == 3 ? -1 : 0); oy <= (DIM == 3 ? 1 : 0); ++oy) {
                T row = 0;
                for (int ox = -1; ox <= 1; ++ox) {
                    const int i = fi + ox, j = fj + oy, k = fk + oz;
                    const int q = DIM == 3 ? i + f.n * (j + f.n * k) : i;
                    const T res = f.b[q] - (f.u[q] - ah * f.d2(f.u, i, j, k));
                    row += w[ox + 1] * res;
                }
                acc += (DIM == 3 ? w[oz + 1] * w[oy + 1] : (T)1) * row;
            }
        c.b[p] = acc;
    });
}

template <int DIM, typename T>
__device__ void prolong_add(const Grid<DIM, T> &c, Grid<DIM, T> &f)
{
    for_points<DIM>(f.n, [&](int p, int i, int j, int k) {
        // 1-based fine index i+1; coarse 1-based (i+1)>>1 and (i+2)>>1, 0-based minus one
        const int i1 = i + 1;
        const int a0 = (i1 >> 1) - 1, a1 = ((i1 + 1) >> 1) - 1;
        auto rowv = [&](int jj, int kk) -> T {
            return (i1 & 1) ? (T)0.5 * (c.at(c.u, a0, jj, kk) + c.at(c.u, a1, jj, kk)) : c.at(c.u, a0, jj, kk);
        };
        T v;
        if (DIM == 3) {
            const int j1 = j + 1, k1 = k + 1;
            const int b0 = (j1 >> 1) - 1, b1 = ((j1 + 1) >> 1) - 1, c0 = (k1 >> 1) - 1, c1 = ((k1 + 1) >> 1) - 1;
            auto planev = [&](int kk) -> T {
                return (j1 & 1) ? (T)0.5 * (rowv(b0, kk) + rowv(b1, kk)) : rowv(b0, kk);
            };
            v = (k1 & 1) ? (T)0.5 * (planev(c0) + planev(c1)) : planev(c0);
        } else {
            v = rowv(0, 0);
        }
        f.u[p] += v;
    });
}

// Exact solve for n in {1, 2} (see the coarsest kernel for the transform).
template <int DIM, typename T>
__device__ void coarsest(Grid<DIM, T> &g, T ah)
{
    if (threadIdx.x + threadIdx.y + threadIdx.z != 0) return;
    if (g.n == 1) {
        g.u[0] = g.b[0] / ((T)1 + (T)(2 * DIM) * ah);
        return;
    }
    if (DIM == 1) {
        const T b1 = g.b[0], b2 = g.b[1];
        const T p = (b1 + b2) / ((T)1 + ah), q = (b1 - b2) / ((T)1 + (T)3 * ah);
        g.u[0] = (T)0.5 * (p + q);
        g.u[1] = (T)0.5 * (p - q);
        return;
    }
    T coef[8];
#pragma unroll
    for (int sgn = 0; sgn < 8; ++sgn) {
        T dot = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool neg = (__builtin_popcount(sgn & q) & 1) != 0;
            dot += neg ? -g.b[q] : g.b[q];
        }
        const int nneg = __builtin_popcount(sgn);
        coef[sgn] = dot / ((T)8 * ((T)1 + ah * (T)(3 + 2 * nneg)));
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        T acc = 0;
#pragma unroll
        for (int sgn = 0; sgn < 8; ++sgn) {
            const bool neg = (__builtin_popcount(sgn & q) & 1) != 0;
            acc += neg ? -coef[sgn] : coef[sgn];
        }
        g.u[q] = acc;
    }
}

template <int DIM, typename T>
__global__ __launch_bounds__(1024) void vcycle_bottom_kernel(Tiling t, double alpha_s, int smoother, double omega,
                                                             int nu1, int nu2, int zero_init, View<T> bg,
                                                             View<T> ug)
{
    extern __shared__ unsigned char smem_raw[];
    unsigned bid = blockIdx.x;
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [](int) { return 1L; })) return;
    qs.item = (int)bid;
    if (mask && !mask[qs.item]) return;
    const int n0 = qs.n;
    const double alpha = qs.par(alpha_s);
    // level table in LDS (a runtime-indexed private array would live in scratch)
    __shared__ int sn[MAXL], snl;
    __shared__ unsigned soff[MAXL];
    __shared__ T sah[MAXL], swi[MAXL];
    const bool lead = threadIdx.x + threadIdx.y + threadIdx.z == 0;
    if (lead) {
        int nl = 0;
        unsigned off = 0;
        for (int n = n0;; n = coarser(n)) {
            sn[nl] = n;
            soff[nl] = off;
            off += (unsigned)((smoother == PFMG_SMOOTH_JACOBI ? 3 : 2) * ipow(n, DIM));
            const double ah = alpha * (double)(n + 1) * (double)(n + 1);
            sah[nl] = (T)ah;
            swi[nl] = (T)(omega / (1.0 + 2.0 * DIM * ah));
            ++nl;
            if (n <= 2 || nl == MAXL) break;
        }
        snl = nl;
    }
    __syncthreads();
    T *base = reinterpret_cast<T *>(smem_raw);
    auto grid = [&](int l) -> Grid<DIM, T> {
        Grid<DIM, T> g;
        const int len = ipow(sn[l], DIM);
        g.n = sn[l];
        g.u = base + soff[l];
        g.b = g.u + len;
        g.t = g.u + 2 * len;
        return g;
    };
    const int nl = snl;
    const T *bsrc = fp(bg, qs);
    T *udst = fp(ug, qs);
    const long sy = row_stride(n0), sz = plane_stride(n0);
    {
        const Grid<DIM, T> top = grid(0);
        for_points<DIM>(n0, [&](int p, int i, int j, int k) {
            const long o = DIM == 3 ? (long)(i + 1) + (long)(j + 1) * sy + (long)(k + 1) * sz : (long)(i + 1);
            top.b[p] = bsrc[o];
            top.u[p] = zero_init ? (T)0 : udst[o];
        });
    }
    __syncthreads();
    if (n0 <= 2) {
        Grid<DIM, T> g0 = grid(0);
        coarsest<DIM, T>(g0, sah[0]);
        __syncthreads();
    } else {
        for (int l = 0; l + 1 < nl; ++l) {
            Grid<DIM, T> gf = grid(l), gc = grid(l + 1);
            smooth<DIM, T>(gf, sah[l], swi[l], smoother, nu1, l > 0 || zero_init);
            resid_restrict<DIM, T>(gf, gc, sah[l]);
            __syncthreads();
        }
        Grid<DIM, T> gb = grid(nl - 1);
        coarsest<DIM, T>(gb, sah[nl - 1]);
        __syncthreads();
        for (int l = nl - 2; l >= 0; --l) {
            Grid<DIM, T> gf = grid(l), gc = grid(l + 1);
            prolong_add<DIM, T>(gc, gf);
            __syncthreads();
            smooth<DIM, T>(gf, sah[l], swi[l], smoother, nu2, false);
        }
    }
    const Grid<DIM, T> top = grid(0);
    for_points<DIM>(n0, [&](int p, int i, int j, int k) {
        const long o = DIM == 3 ? (long)(i + 1) + (long)(j + 1) * sy + (long)(k + 1) * sz : (long)(i + 1);
        udst[o] = top.u[p];
    });
}

}  // namespace

namespace k {

size_t vcycle_bottom_lds(int n0, int dim, int smoother, size_t elem)
{
    size_t total = 0;
    for (int n = n0;; n = coarser(n)) {
        total += (size_t)(smoother == PFMG_SMOOTH_JACOBI ? 3 : 2) * ipow(n, dim) * elem;
        if (n <= 2) break;
    }
    return total;
}

template <typename T>
hipError_t vcycle_bottom(const Tiling &t, double alpha, int smoother, double omega, int nu1, int nu2, bool zero_init,
                         View<T> b, View<T> u, hipStream_t s)
{
    long items = 0;
    size_t lds = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        items += t.seg_count(sg);
        lds = std::max(lds, vcycle_bottom_lds(t.seg_n(sg), t.dim, smoother, sizeof(T)));
    }
    if (items == 0) return hipSuccess;
    if (lds > BOTTOM_LDS_MAX) return hipErrorInvalidValue;
    // workgroup shape (x, y, z threads; x fastest) for the largest grid of
    // the launch: every thread owns a few points of each pass
    static const int shape = [] {
        const char *e = getenv("PFMG_BOTTOM_THREADS");
        return e ? atoi(e) : 1024;
    }();
    const dim3 blk = shape == 256 ? dim3(8, 8, 4) : shape == 512 ? dim3(16, 8, 4) : dim3(16, 16, 4);
    if (t.dim == 3)
        vcycle_bottom_kernel<3, T><<<(unsigned)items, blk, lds, s>>>(t, alpha, smoother, omega, nu1, nu2,
                                                                                 zero_init ? 1 : 0, b, u);
    else
        vcycle_bottom_kernel<1, T><<<(unsigned)items, dim3(BT, 1, 1), lds, s>>>(t, alpha, smoother, omega, nu1, nu2,
                                                                                zero_init ? 1 : 0, b, u);
    return hipGetLastError();
}

template hipError_t vcycle_bottom<double>(const Tiling &, double, int, double, int, int, bool, View<double>,
                                          View<double>, hipStream_t);
template hipError_t vcycle_bottom<float>(const Tiling &, double, int, double, int, int, bool, View<float>,
                                         View<float>, hipStream_t);

}  // namespace k
}  // namespace pfmg
