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
// Dirichlet data.  Each level holds u, b and a third array t (Jacobi's
// target, and the residual before restriction), so that every residual is
// computed once rather than once per coarse neighbour.
//
// The kernel is latency-bound (a single-field coarse solve sits on the
// serial coarse chain of PFASST), so passes spread their points evenly over
// all threads: a red-black colour pass visits only its own colour.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/pfmg.h"
#include "kernels.h"

namespace pfmg {
namespace {

constexpr int MAXL = 16;
constexpr int BT = 1024;          // 3D: 16 x 16 x 4 threads; 1D: 1024 x 1 x 1

// Visit every point of an n^DIM grid: coordinates come from the thread
// index (no integer division), p is the dense index.  Rows of 16 threads:
// the global loads and stores of the top grid.
template <int DIM, class F>
__device__ inline void for_points(int n, F f)
{
    if (DIM == 3) {
        for (int k = threadIdx.z; k < n; k += 4)
            for (int j = threadIdx.y; j < n; j += 16)
                for (int i = threadIdx.x; i < n; i += 16) f(i + n * (j + n * k), i, j, k);
    } else {
        for (int i = threadIdx.x; i < n; i += BT) f(i, i, 0, 0);
    }
}

template <int DIM>
__device__ inline int flat_tid()
{
    return DIM == 3 ? (int)(threadIdx.x + 16 * (threadIdx.y + 16 * threadIdx.z)) : (int)threadIdx.x;
}

// Every point of an n^DIM grid, BT points per round.  3D grids with n <= 8
// take 8 x 16 x 8 points per round from the 16 x 16 x 4 thread block (x
// lanes split in two z halves), n <= 16 take 16 x 16 x 4; both without
// integer division.  Larger grids go in dense index order.
template <int DIM, class F>
__device__ inline void for_flat(int n, F f)
{
    if (DIM == 3 && n <= 8) {
        const int i = threadIdx.x & 7, j = threadIdx.y;
        if (i < n && j < n)
            for (int k = 2 * threadIdx.z + (threadIdx.x >> 3); k < n; k += 8) f(i + n * (j + n * k), i, j, k);
        return;
    }
    if (DIM == 3 && n <= 16) {
        if (threadIdx.x < n && threadIdx.y < n)
            for (int k = threadIdx.z; k < n; k += 4) {
                const int i = threadIdx.x, j = threadIdx.y;
                f(i + n * (j + n * k), i, j, k);
            }
        return;
    }
    if (DIM == 3) {
        const int nn = n * n;
        for (int p = flat_tid<DIM>(); p < nn * n; p += BT) {
            const int k = p / nn, r = p - k * nn;
            const int j = r / n, i = r - j * n;
            f(p, i, j, k);
        }
    } else {
        for (int i = flat_tid<DIM>(); i < n; i += BT) f(i, i, 0, 0);
    }
}

// The points of one colour: 1-based parity (i + j + k + 3) & 1 == colour,
// i.e. i runs over every other point of its row, starting where the row's
// parity puts the colour.
template <int DIM, class F>
__device__ inline void for_colour(int n, int colour, F f)
{
    const int h = (n + 1) / 2;
    if (DIM == 3 && n <= 16) {
        // 8 x 16 x 8 (i/2, j, k) slots per round, no integer division
        const int i2 = threadIdx.x & 7, j = threadIdx.y;
        if (i2 < h && j < n)
            for (int k = 2 * threadIdx.z + (threadIdx.x >> 3); k < n; k += 8) {
                const int i = 2 * i2 + ((colour + j + k + 1) & 1);
                if (i < n) f(i + n * (j + n * k), i, j, k);
            }
        return;
    }
    if (DIM == 3) {
        const int hn = h * n;
        for (int q = flat_tid<DIM>(); q < hn * n; q += BT) {
            const int k = q / hn, r = q - k * hn;
            const int j = r / h, i2 = r - j * h;
            const int i = 2 * i2 + ((colour + j + k + 1) & 1);
            if (i < n) f(i + n * (j + n * k), i, j, k);
        }
    } else {
        for (int i2 = flat_tid<DIM>(); i2 < h; i2 += BT) {
            const int i = 2 * i2 + ((colour + 1) & 1);
            if (i < n) f(i, i, 0, 0);
        }
    }
}

__host__ __device__ inline int ipow(int n, int dim) { return dim == 3 ? n * n * n : n; }

template <int DIM, typename T>
struct Grid {
    T *u, *b, *t;
    int n;
    // Value at (i, j, k), zero outside the grid.  The read is unconditional
    // (from point 0 when outside) and the zero is a select: a branch per
    // neighbour would serialise the LDS reads of a stencil.
    __device__ T at(const T *a, int i, int j, int k) const
    {
        const bool ok = (unsigned)i < (unsigned)n &&
                        (DIM == 1 || ((unsigned)j < (unsigned)n && (unsigned)k < (unsigned)n));
        const T v = a[ok ? (DIM == 3 ? i + n * (j + n * k) : i) : 0];
        return ok ? v : (T)0;
    }
    __device__ void coords(int p, int &i, int &j, int &k) const
    {
        if (DIM == 3) { i = p % n; j = (p / n) % n; k = p / (n * n); }
        else { i = p; j = k = 0; }
    }
    // Neighbour of interior point p at offset off when `ok`, else zero.
    __device__ T nb(const T *a, int p, int off, bool ok) const
    {
        const T v = a[ok ? p + off : p];
        return ok ? v : (T)0;
    }
    __device__ T d2(const T *a, int i, int j, int k) const
    {
        const int p = DIM == 3 ? i + n * (j + n * k) : i;
        const T c = a[p];
        T s = nb(a, p, -1, i > 0) + nb(a, p, 1, i < n - 1);
        if (DIM == 3)
            s += (nb(a, p, -n, j > 0) + nb(a, p, n, j < n - 1)) + (nb(a, p, -n * n, k > 0) + nb(a, p, n * n, k < n - 1));
        return s - (T)(2 * DIM) * c;
    }
};

template <int DIM, typename T>
__device__ void smooth(Grid<DIM, T> &g, T ah, T winv, int smoother, int sweeps, bool from_zero)
{
    if (sweeps == 0 && from_zero) {
        for_flat<DIM>(g.n, [&](int p, int, int, int) { g.u[p] = (T)0; });
        __syncthreads();
        return;
    }
    for (int s = 0; s < sweeps; ++s) {
        const bool z = s == 0 && from_zero;
        if (smoother == PFMG_SMOOTH_RBGS) {
            if (z) {
                // red pass from u = 0: red points winv b, black points 0
                for_flat<DIM>(g.n, [&](int p, int i, int j, int k) {
                    const int par = (DIM == 3 ? (i + j + k + 3) : (i + 1)) & 1;
                    g.u[p] = par == 0 ? winv * g.b[p] : (T)0;
                });
                __syncthreads();
            }
            for (int colour = z ? 1 : 0; colour < 2; ++colour) {
                for_colour<DIM>(g.n, colour, [&](int p, int i, int j, int k) {
                    const T uc = g.u[p];
                    g.u[p] = uc + winv * (g.b[p] - (uc - ah * g.d2(g.u, i, j, k)));
                });
                __syncthreads();
            }
        } else {
            for_flat<DIM>(g.n, [&](int p, int i, int j, int k) {
                if (z) {
                    g.t[p] = winv * g.b[p];
                } else {
                    const T uc = g.u[p];
                    g.t[p] = uc + winv * (g.b[p] - (uc - ah * g.d2(g.u, i, j, k)));
                }
            });
            __syncthreads();
            for_flat<DIM>(g.n, [&](int p, int, int, int) { g.u[p] = g.t[p]; });
            __syncthreads();
        }
    }
}

// Coarse b = full weighting of the fine residual b - (u - ah L u): the
// residual of every fine point goes to f.t first (fine points 2I, 2I+1,
// 2I+2 of each coarse point I, 0-based, all lie inside the fine grid).
template <int DIM, typename T>
__device__ void resid_restrict(Grid<DIM, T> &f, Grid<DIM, T> &c, T ah)
{
    for_flat<DIM>(f.n, [&](int p, int i, int j, int k) { f.t[p] = f.b[p] - (f.u[p] - ah * f.d2(f.u, i, j, k)); });
    __syncthreads();
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    for_flat<DIM>(c.n, [&](int p, int I, int J, int K) {
        const int fi = 2 * I + 1, fj = DIM == 3 ? 2 * J + 1 : 0, fk = DIM == 3 ? 2 * K + 1 : 0;
        T acc = 0;
#pragma unroll
        for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
#pragma unroll
            for (int oy = (DIM == 3 ? -1 : 0); oy <= (DIM == 3 ? 1 : 0); ++oy) {
                T row = 0;
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                    const int q = DIM == 3 ? (fi + ox) + f.n * ((fj + oy) + f.n * (fk + oz)) : fi + ox;
                    row += w[ox + 1] * f.t[q];
                }
                acc += (DIM == 3 ? w[oz + 1] * w[oy + 1] : (T)1) * row;
            }
        c.b[p] = acc;
    });
}

template <int DIM, typename T>
__device__ void prolong_add(const Grid<DIM, T> &c, Grid<DIM, T> &f)
{
    // fine 1-based index x1: even sits on coarse x1/2, odd between
    // (x1-1)/2 and (x1+1)/2 (1-based; 0 and nc+1 are the zero boundary).
    // All eight coarse values are read unconditionally (the two indices
    // coincide on an even axis) and combined with selects, so the LDS
    // reads issue together: per axis 0.5 (lo + hi) when odd, lo when even.
    for_flat<DIM>(f.n, [&](int p, int i, int j, int k) {
        const int i1 = i + 1;
        const int a0 = (i1 >> 1) - 1, a1 = ((i1 + 1) >> 1) - 1;
        const bool ox = (i1 & 1) != 0;
        auto rowv = [&](int jj, int kk) -> T {
            const T x0 = c.at(c.u, a0, jj, kk), x1 = c.at(c.u, a1, jj, kk);
            const T h = (T)0.5 * (x0 + x1);
            return ox ? h : x0;
        };
        T v;
        if (DIM == 3) {
            const int j1 = j + 1, k1 = k + 1;
            const int b0 = (j1 >> 1) - 1, b1 = ((j1 + 1) >> 1) - 1, c0 = (k1 >> 1) - 1, c1 = ((k1 + 1) >> 1) - 1;
            const bool oy = (j1 & 1) != 0, oz = (k1 & 1) != 0;
            const T r00 = rowv(b0, c0), r10 = rowv(b1, c0), r01 = rowv(b0, c1), r11 = rowv(b1, c1);
            const T p0h = (T)0.5 * (r00 + r10), p1h = (T)0.5 * (r01 + r11);
            const T p0 = oy ? p0h : r00, p1 = oy ? p1h : r01;
            const T vh = (T)0.5 * (p0 + p1);
            v = oz ? vh : p0;
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
    // thread l fills level l (levels: n0, coarser(n0), ... down to n <= 2)
    const int tid = flat_tid<DIM>();
    if (tid < MAXL) {
        int n = n0, l = 0;
        unsigned off = 0;
        while (l < tid && n > 2) {
            off += (unsigned)(3 * ipow(n, DIM));
            n = coarser(n);
            ++l;
        }
        if (l == tid) {
            sn[l] = n;
            soff[l] = off;
            const double ah = alpha * (double)(n + 1) * (double)(n + 1);
            sah[l] = (T)ah;
            swi[l] = (T)(omega / (1.0 + 2.0 * DIM * ah));
            if (n <= 2 || l == MAXL - 1) snl = l + 1;
        }
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

size_t bottom_lds_max()
{
    static const size_t cap = [] {
        int dev = 0, bytes = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            bytes = 64 * 1024;
        return (size_t)std::max(bytes, 64 * 1024) - 1024;
    }();
    return cap;
}

size_t vcycle_bottom_lds(int n0, int dim, int smoother, size_t elem)
{
    size_t total = 0;
    for (int n = n0;; n = coarser(n)) {
        total += (size_t)3 * ipow(n, dim) * elem;
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
    if (lds > bottom_lds_max()) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        // above the default dynamic-LDS limit: raise it once per kernel
        static const hipError_t e3 = hipFuncSetAttribute((const void *)vcycle_bottom_kernel<3, T>,
                                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                                         (int)bottom_lds_max());
        static const hipError_t e1 = hipFuncSetAttribute((const void *)vcycle_bottom_kernel<1, T>,
                                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                                         (int)bottom_lds_max());
        if ((t.dim == 3 ? e3 : e1) != hipSuccess) return t.dim == 3 ? e3 : e1;
    }
    if (t.dim == 3)
        vcycle_bottom_kernel<3, T><<<(unsigned)items, dim3(16, 16, 4), lds, s>>>(t, alpha, smoother, omega, nu1, nu2,
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
