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
#include <cstdlib>

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


// ---------------------------------------------------------------------------
// The same V-cycle for the case the big-grid V-cycles hand down (3D, top grid
// 15^3, red-black smoother): levels 15, 7, 3, 1 with compile-time sizes, so
// every loop over points is unrolled and its index arithmetic folded.  A pass
// first reads everything it needs (its points' neighbours have the other
// colour, or live in another array), then writes, so the LDS reads of all
// its points are in flight together; the level constants live in registers.
// The arithmetic is that of the generic kernel above, term for term.
namespace b15 {

constexpr int N0 = 15, N1 = 7, N2 = 3;
// dense level arrays u, b, t of each level, one after the other in LDS
constexpr int OFF1 = 3 * N0 * N0 * N0, OFF2 = OFF1 + 3 * N1 * N1 * N1, OFF3 = OFF2 + 3 * N2 * N2 * N2;
constexpr int LDS_ELEMS = OFF3 + 3;

// One point of an N^3 grid per slot; rounds of 16 x 16 x 4 slots for
// 8 < N <= 16, of 8 x 16 x 8 for N <= 8 (as the generic kernel visits them).
template <int N>
struct All {
    static constexpr int R = N > 8 ? (N + 3) / 4 : 1;
    __device__ static void at(int r, int &i, int &j, int &k, bool &ok)
    {
        if (N > 8) {
            i = threadIdx.x; j = threadIdx.y; k = threadIdx.z + 4 * r;
        } else {
            i = threadIdx.x & 7; j = threadIdx.y; k = 2 * threadIdx.z + (threadIdx.x >> 3);
        }
        ok = i < N && j < N && k < N;
    }
};

// One point of colour c (1-based parity (i + j + k + 3) & 1 == c) per slot:
// i / 2 from the low x lanes, rounds of 8 x 16 x 8 slots.
template <int N>
struct Colour {
    static constexpr int H = (N + 1) / 2, R = (N + 7) / 8;
    __device__ static void at(int r, int c, int &i, int &j, int &k, bool &ok)
    {
        const int i2 = threadIdx.x & 7;
        j = threadIdx.y;
        k = 2 * threadIdx.z + (threadIdx.x >> 3) + 8 * r;
        i = 2 * i2 + ((c + j + k + 1) & 1);
        ok = i2 < H && j < N && k < N && i < N;
    }
};

template <int N>
__device__ inline int idx(int i, int j, int k) { return i + N * (j + N * k); }

// Laplacian numerator of point (i, j, k) (inside the grid): neighbours
// outside read the point itself and are replaced by the zero boundary.
template <int N, typename T>
__device__ inline T d2(const T *a, int i, int j, int k)
{
    const int p = idx<N>(i, j, k);
    auto nb = [&](int off, bool in) { const T v = a[in ? p + off : p]; return in ? v : (T)0; };
    const T c = a[p];
    T s = nb(-1, i > 0) + nb(1, i < N - 1);
    s += (nb(-N, j > 0) + nb(N, j < N - 1)) + (nb(-N * N, k > 0) + nb(N * N, k < N - 1));
    return s - (T)6 * c;
}

// Gauss-Seidel update of colour c in place.
template <int N, typename T>
__device__ inline void rb_pass(T *u, const T *b, T ah, T winv, int c)
{
    constexpr int R = Colour<N>::R;
    T v[R];
    int pp[R];
    bool okr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i, j, k;
        bool ok;
        Colour<N>::at(r, c, i, j, k, ok);
        if (!ok) i = j = k = 0;
        const int p = idx<N>(i, j, k);
        const T uc = u[p];
        v[r] = uc + winv * (b[p] - (uc - ah * d2<N>(u, i, j, k)));
        pp[r] = p;
        okr[r] = ok;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (okr[r]) u[pp[r]] = v[r];
    __syncthreads();
}

// RB-GS sweeps on a small grid (N <= 8: one slot round per colour); from
// zero the first red pass is winv b on red points, 0 on black ones.
template <int N, typename T>
__device__ inline void smooth_pt(T *u, const T *b, T ah, T winv, int sweeps, bool from_zero)
{
    if (sweeps == 0 && from_zero) {
#pragma unroll
        for (int r = 0; r < All<N>::R; ++r) {
            int i, j, k;
            bool ok;
            All<N>::at(r, i, j, k, ok);
            if (ok) u[idx<N>(i, j, k)] = (T)0;
        }
        __syncthreads();
        return;
    }
    for (int sw = 0; sw < sweeps; ++sw) {
        const bool z = sw == 0 && from_zero;
        if (z) {
            constexpr int R = All<N>::R;
            T v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                int i, j, k;
                bool ok;
                All<N>::at(r, i, j, k, ok);
                const T bv = b[ok ? idx<N>(i, j, k) : 0];
                v[r] = ((i + j + k + 3) & 1) == 0 ? winv * bv : (T)0;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                int i, j, k;
                bool ok;
                All<N>::at(r, i, j, k, ok);
                if (ok) u[idx<N>(i, j, k)] = v[r];
            }
            __syncthreads();
        } else {
            rb_pass<N>(u, b, ah, winv, 0);
        }
        rb_pass<N>(u, b, ah, winv, 1);
    }
}

// RB-GS sweeps; from zero the first red pass is winv b on red points, 0 on
// black ones.  A thread visits the same points (slot r of colour c) in every
// pass, so it keeps their b and their current u in registers: a pass reads
// only the six neighbours from LDS.  The arithmetic is that of the generic
// kernel (the centre value is the same number, held in a register).
template <int N, typename T>
__device__ inline void smooth(T *u, const T *b, T ah, T winv, int sweeps, bool from_zero)
{
    if constexpr (N <= 8) {
        // small grids: the registers would cost more than the LDS reads
        smooth_pt<N>(u, b, ah, winv, sweeps, from_zero);
        return;
    }
    constexpr int R = Colour<N>::R;
    int ci[2][R], cj[2][R], ck[2][R], pp[2][R];
    bool okr[2][R];
    T bb[2][R], uu[2][R];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int i, j, k;
            bool ok;
            Colour<N>::at(r, c, i, j, k, ok);
            if (!ok) i = j = k = 0;
            ci[c][r] = i; cj[c][r] = j; ck[c][r] = k;
            pp[c][r] = idx<N>(i, j, k);
            okr[c][r] = ok;
            bb[c][r] = b[pp[c][r]];
            uu[c][r] = from_zero ? (T)0 : u[pp[c][r]];
        }
    if (sweeps == 0) {
        if (from_zero) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (okr[c][r]) u[pp[c][r]] = (T)0;
        }
        __syncthreads();
        return;
    }
    auto pass = [&](int c) {
        T v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = ci[c][r], j = cj[c][r], k = ck[c][r], p = pp[c][r];
            auto nb = [&](int off, bool in) { const T x = u[in ? p + off : p]; return in ? x : (T)0; };
            T sn = nb(-1, i > 0) + nb(1, i < N - 1);
            sn += (nb(-N, j > 0) + nb(N, j < N - 1)) + (nb(-N * N, k > 0) + nb(N * N, k < N - 1));
            const T uc = uu[c][r];
            const T d2 = sn - (T)6 * uc;
            v[r] = uc + winv * (bb[c][r] - (uc - ah * d2));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uu[c][r] = v[r];
            if (okr[c][r]) u[pp[c][r]] = v[r];
        }
        __syncthreads();
    };
    for (int sw = 0; sw < sweeps; ++sw) {
        if (sw == 0 && from_zero) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    uu[c][r] = c == 0 ? winv * bb[c][r] : (T)0;
                    if (okr[c][r]) u[pp[c][r]] = uu[c][r];
                }
            __syncthreads();
        } else {
            pass(0);
        }
        pass(1);
    }
}

// Fine residual into t, then coarse b = its full weighting.
template <int NF, int NC, typename T>
__device__ inline void resid_restrict(const T *u, const T *b, T *t, T *bc, T ah)
{
    constexpr int R = All<NF>::R;
    T v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i, j, k;
        bool ok;
        All<NF>::at(r, i, j, k, ok);
        if (!ok) i = j = k = 0;
        const int p = idx<NF>(i, j, k);
        v[r] = b[p] - (u[p] - ah * d2<NF>(u, i, j, k));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i, j, k;
        bool ok;
        All<NF>::at(r, i, j, k, ok);
        if (ok) t[idx<NF>(i, j, k)] = v[r];
    }
    __syncthreads();
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
#pragma unroll
    for (int r = 0; r < All<NC>::R; ++r) {
        int I, J, K;
        bool ok;
        All<NC>::at(r, I, J, K, ok);
        if (!ok) I = J = K = 0;
        const int fi = 2 * I + 1, fj = 2 * J + 1, fk = 2 * K + 1;
        T acc = 0;
#pragma unroll
        for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy) {
                T row = 0;
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) row += w[ox + 1] * t[idx<NF>(fi + ox, fj + oy, fk + oz)];
                acc += w[oz + 1] * w[oy + 1] * row;
            }
        if (ok) bc[idx<NC>(I, J, K)] = acc;
    }
    __syncthreads();
}

// Fine u += d-linear interpolation of the coarse u (as prolong_add above),
// point by point (the small levels).
template <int NC, int NF, typename T>
__device__ inline void prolong_pt(const T *uc, T *uf)
{
    auto at = [&](int i, int j, int k) -> T {
        const bool ok = (unsigned)i < (unsigned)NC && (unsigned)j < (unsigned)NC && (unsigned)k < (unsigned)NC;
        const T v = uc[ok ? idx<NC>(i, j, k) : 0];
        return ok ? v : (T)0;
    };
    constexpr int R = All<NF>::R;
    T v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i, j, k;
        bool ok;
        All<NF>::at(r, i, j, k, ok);
        if (!ok) i = j = k = 0;
        const int i1 = i + 1, j1 = j + 1, k1 = k + 1;
        const int a0 = (i1 >> 1) - 1, a1 = ((i1 + 1) >> 1) - 1;
        const int b0 = (j1 >> 1) - 1, b1 = ((j1 + 1) >> 1) - 1, c0 = (k1 >> 1) - 1, c1 = ((k1 + 1) >> 1) - 1;
        const bool ox = (i1 & 1) != 0, oy = (j1 & 1) != 0, oz = (k1 & 1) != 0;
        auto rowv = [&](int jj, int kk) -> T {
            const T x0 = at(a0, jj, kk), x1 = at(a1, jj, kk);
            const T h = (T)0.5 * (x0 + x1);
            return ox ? h : x0;
        };
        const T r00 = rowv(b0, c0), r10 = rowv(b1, c0), r01 = rowv(b0, c1), r11 = rowv(b1, c1);
        const T p0h = (T)0.5 * (r00 + r10), p1h = (T)0.5 * (r01 + r11);
        const T p0 = oy ? p0h : r00, p1 = oy ? p1h : r01;
        const T vh = (T)0.5 * (p0 + p1);
        v[r] = uf[idx<NF>(i, j, k)] + (oz ? vh : p0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i, j, k;
        bool ok;
        All<NF>::at(r, i, j, k, ok);
        if (ok) uf[idx<NF>(i, j, k)] = v[r];
    }
    __syncthreads();
}

// Fine u += d-linear interpolation of the coarse u (as prolong_add above),
// by coarse cells: cell (cx, cy, cz), 0 <= c <= NC, holds the fine points
// with 1-based indices 2c and 2c + 1 on each axis (those inside the grid),
// whose coarse neighbours are the cell's corners c and c + 1 (1-based; 0
// and NC + 1 are the zero boundary).  A thread takes the cell's fine points
// of one z parity: it reads the cell's 4 (even z) or 8 (odd z) corners once
// and combines them with the same selects as the point formula.
template <int NC, int NF, typename T>
__device__ inline void prolong_add(const T *uc, T *uf)
{
    if constexpr (NC < 7) {
        prolong_pt<NC, NF>(uc, uf);
        return;
    }
    constexpr int C = NC + 1, CELLS = C * C * C;
    static_assert(NF == 2 * NC + 1 && 2 * CELLS <= 1024, "cell mapping");
    auto at = [&](int i, int j, int k) -> T {
        const bool ok = (unsigned)i < (unsigned)NC && (unsigned)j < (unsigned)NC && (unsigned)k < (unsigned)NC;
        const T v = uc[ok ? idx<NC>(i, j, k) : 0];
        return ok ? v : (T)0;
    };
    const int tid = (int)(threadIdx.x + 16 * (threadIdx.y + 16 * threadIdx.z));
    const bool act = tid < 2 * CELLS;
    const int zp = tid / CELLS, rem = tid - zp * CELLS;
    const int cx = rem % C, cy = (rem / C) % C, cz = rem / (C * C);
    const int k1 = 2 * cz + zp;   // 1-based fine z of this thread's points
    const bool oz = zp != 0;
    // corners X[a][b][c]: x index cx - 1 + a, y index cy - 1 + b (0-based),
    // z the point's lower (c = 0) and, for odd z, upper (c = 1) coarse plane
    T X[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            X[a][bb][0] = at(cx - 1 + a, cy - 1 + bb, cz - 1);
            X[a][bb][1] = oz ? at(cx - 1 + a, cy - 1 + bb, cz) : X[a][bb][0];
        }
    T v[4], fv[4];
    int pp[4];
    bool okp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i1 = 2 * cx + (q & 1), j1 = 2 * cy + (q >> 1);
        okp[q] = act && i1 >= 1 && i1 <= NF && j1 >= 1 && j1 <= NF && k1 >= 1 && k1 <= NF;
        pp[q] = okp[q] ? idx<NF>(i1 - 1, j1 - 1, k1 - 1) : 0;
        fv[q] = uf[pp[q]];
        const bool ox = (q & 1) != 0, oy = (q >> 1) != 0;
        auto rowv = [&](int bb, int c) -> T {
            const T x0 = X[0][bb][c], x1 = X[ox ? 1 : 0][bb][c];
            const T h = (T)0.5 * (x0 + x1);
            return ox ? h : x0;
        };
        const T r00 = rowv(0, 0), r10 = rowv(oy ? 1 : 0, 0), r01 = rowv(0, 1), r11 = rowv(oy ? 1 : 0, 1);
        const T p0h = (T)0.5 * (r00 + r10), p1h = (T)0.5 * (r01 + r11);
        const T p0 = oy ? p0h : r00, p1 = oy ? p1h : r01;
        const T vh = (T)0.5 * (p0 + p1);
        v[q] = oz ? vh : p0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (okp[q]) uf[pp[q]] = fv[q] + v[q];
    __syncthreads();
}

}  // namespace b15

template <typename T>
__global__ __launch_bounds__(1024) void vcycle_bottom15_kernel(Tiling t, double alpha_s, double omega, int nu1, int nu2,
                                                               int zero_init, View<T> bg, View<T> ug)
{
    using namespace b15;
    extern __shared__ unsigned char smem_raw[];
    unsigned bid = blockIdx.x;
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [](int) { return 1L; })) return;
    qs.item = (int)bid;
    if (mask && !mask[qs.item]) return;
    const double alpha = qs.par(alpha_s);
    // per level: ah = alpha (n + 1)^2, winv = omega / (1 + 6 ah)
    const double a0 = alpha * 256.0, a1 = alpha * 64.0, a2 = alpha * 16.0, a3 = alpha * 4.0;
    const T ah0 = (T)a0, ah1 = (T)a1, ah2 = (T)a2, ah3 = (T)a3;
    const T wi0 = (T)(omega / (1.0 + 6.0 * a0)), wi1 = (T)(omega / (1.0 + 6.0 * a1)),
            wi2 = (T)(omega / (1.0 + 6.0 * a2));
    T *base = reinterpret_cast<T *>(smem_raw);
    T *u0 = base, *b0 = u0 + N0 * N0 * N0, *t0 = b0 + N0 * N0 * N0;
    T *u1 = base + OFF1, *b1 = u1 + N1 * N1 * N1, *t1 = b1 + N1 * N1 * N1;
    T *u2 = base + OFF2, *b2 = u2 + N2 * N2 * N2, *t2 = b2 + N2 * N2 * N2;
    T *u3 = base + OFF3, *b3 = u3 + 1;
    const T *bsrc = fp(bg, qs);
    T *udst = fp(ug, qs);
    constexpr int sy = N0 + 1, sz = (N0 + 1) * (N0 + 2);
    // the top grid: every global load issued before the first LDS store
    // (slots outside the grid read element 0, a halo word)
    {
        constexpr int R = All<N0>::R;
        T bv[R], uv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int i, j, k;
            bool ok;
            All<N0>::at(r, i, j, k, ok);
            const int o = ok ? (i + 1) + (j + 1) * sy + (k + 1) * sz : 0;
            bv[r] = bsrc[o];
            uv[r] = zero_init ? (T)0 : udst[o];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int i, j, k;
            bool ok;
            All<N0>::at(r, i, j, k, ok);
            if (ok) {
                b0[idx<N0>(i, j, k)] = bv[r];
                u0[idx<N0>(i, j, k)] = uv[r];
            }
        }
    }
    __syncthreads();
    smooth<N0>(u0, b0, ah0, wi0, nu1, zero_init != 0);
    resid_restrict<N0, N1>(u0, b0, t0, b1, ah0);
    smooth<N1>(u1, b1, ah1, wi1, nu1, true);
    resid_restrict<N1, N2>(u1, b1, t1, b2, ah1);
    smooth<N2>(u2, b2, ah2, wi2, nu1, true);
    resid_restrict<N2, 1>(u2, b2, t2, b3, ah2);
    if (threadIdx.x + threadIdx.y + threadIdx.z == 0) u3[0] = b3[0] / ((T)1 + (T)6 * ah3);
    __syncthreads();
    prolong_add<1, N2>(u3, u2);
    smooth<N2>(u2, b2, ah2, wi2, nu2, false);
    prolong_add<N2, N1>(u2, u1);
    smooth<N1>(u1, b1, ah1, wi1, nu2, false);
    prolong_add<N1, N0>(u1, u0);
    smooth<N0>(u0, b0, ah0, wi0, nu2, false);
#pragma unroll
    for (int r = 0; r < All<N0>::R; ++r) {
        int i, j, k;
        bool ok;
        All<N0>::at(r, i, j, k, ok);
        if (ok) udst[(i + 1) + (j + 1) * sy + (k + 1) * sz] = u0[idx<N0>(i, j, k)];
    }
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
    // 3D red-black from a 15^3 top: the kernel with compile-time levels
    // (PFMG_BOTTOM15=0 keeps the generic one)
    static const bool use15 = [] {
        const char *e = getenv("PFMG_BOTTOM15");
        return !(e && atoi(e) == 0);
    }();
    bool all15 = t.dim == 3 && smoother == PFMG_SMOOTH_RBGS && use15;
    for (int sg = 0; sg < t.nseg; ++sg) all15 = all15 && t.seg_n(sg) == b15::N0;
    if (all15) {
        const size_t l15 = (size_t)b15::LDS_ELEMS * sizeof(T);
        if (l15 > 64 * 1024) {
            static const hipError_t e15 = hipFuncSetAttribute((const void *)vcycle_bottom15_kernel<T>,
                                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                                              (int)bottom_lds_max());
            if (e15 != hipSuccess) return e15;
        }
        vcycle_bottom15_kernel<T><<<(unsigned)items, dim3(16, 16, 4), l15, s>>>(t, alpha, omega, nu1, nu2,
                                                                                zero_init ? 1 : 0, b, u);
        return hipGetLastError();
    }
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
