// Geometric multigrid kernels for (I - alpha L_h) u = b on gfx950.
//
// The node solves of the SDC sweep (eq. SDCcompactLIII, alpha = nu dt_m)
// are done with V-cycles: pre/post smoothing, residual, full-weighting
// restriction, linear interpolation (Sec. 4.1.1, Sec. 4.2.1).  Coarse
// operators are re-discretised on h_{l+1} = 2 h_l with the same alpha;
// grids with n in {1, 2} are solved exactly.
//
// All kernels are memory-bound stencils, no matrix cores.  FP64 and FP32
// instances serve the plain and the mixed-precision forms.  Every launch may
// span several segments (fields of different grids, per-field alpha), so the
// uneven problems of a batch share one launch per multigrid level.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>

#include "kernels.h"

namespace pfmg {
namespace {

// Coefficients of (I - alpha L_h) on grid n: ah = alpha / h^2 and the
// smoother weight omega / diag(H), formed in double.
__host__ __device__ inline double ah_d(double alpha, int n) { return alpha * (double)(n + 1) * (double)(n + 1); }
__host__ __device__ inline double winv_d(double alpha, double omega, int n, int dim)
{
    return omega / (1.0 + 2.0 * dim * ah_d(alpha, n));
}

// ------------------------------------------------------ point kernels
// One thread per point (used in 1D and for small 3D grids).
template <int DIM, typename T, typename TO>
__global__ __launch_bounds__(BLOCK) void resid_kernel(Tiling t, double alpha, View<T> b, View<T> u, View<TO> r)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    const T ah = (T)ah_d(q.par(alpha), q.n);
    const T *uu = fp(u, q);
    const T lap = d2sum<DIM>(uu, c, row_stride(q.n), plane_stride(q.n));
    fp(r, q)[c] = (TO)(fp(b, q)[c] - (uu[c] - ah * lap));
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void jacobi_kernel(Tiling t, double alpha, double omega, View<T> b, View<T> u,
                                                       View<T> out)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    const double a = q.par(alpha);
    const T ah = (T)ah_d(a, q.n), winv = (T)winv_d(a, omega, q.n, DIM);
    const T *uu = fp(u, q);
    const T lap = d2sum<DIM>(uu, c, row_stride(q.n), plane_stride(q.n));
    const T res = fp(b, q)[c] - (uu[c] - ah * lap);
    fp(out, q)[c] = uu[c] + winv * res;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void jacobi_zero_kernel(Tiling t, double alpha, double omega, View<T> b,
                                                            View<T> out)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    const T winv = (T)winv_d(q.par(alpha), omega, q.n, DIM);
    fp(out, q)[c] = winv * fp(b, q)[c];
}

// Red (colour 0: 1-based i+j+k even) or black points, in place.
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void rbgs_kernel(Tiling t, double alpha, double omega, int colour, View<T> b,
                                                     View<T> u)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    const int par = (DIM == 3 ? (i + j + k) : i) & 1;
    if (par != colour) return;
    const double a = q.par(alpha);
    const T ah = (T)ah_d(a, q.n), winv = (T)winv_d(a, omega, q.n, DIM);
    T *uu = fp(u, q);
    const T lap = d2sum<DIM>(uu, c, row_stride(q.n), plane_stride(q.n));
    const T res = fp(b, q)[c] - (uu[c] - ah * lap);
    uu[c] = uu[c] + winv * res;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void rbgs_zero_red_kernel(Tiling t, double alpha, double omega, View<T> b,
                                                              View<T> u)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    const T winv = (T)winv_d(q.par(alpha), omega, q.n, DIM);
    const int par = (DIM == 3 ? (i + j + k) : i) & 1;
    fp(u, q)[c] = par == 0 ? winv * fp(b, q)[c] : (T)0;
}

// ---------------------------------------------------------- restriction
// Launched on the coarse grids (q.n = coarse n); the fine grid is
// 2 (nc + 1) - 1.  Coarse point J (1-based) sits on fine point 2J.
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void restrict_kernel(Tiling t, View<T> r, View<T> bc)
{
    Pt q; int I, J, K; long cc;
    if (!tile_point<DIM>(t, q, I, J, K, cc)) return;
    const int nf = 2 * (q.n + 1) - 1;
    const T *rr = fp(r, q);
    const long sy = row_stride(nf), sz = plane_stride(nf);
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    T acc = 0;
    if (DIM == 3) {
        const long f = 2L * I + 2L * J * sy + 2L * K * sz;
        for (int c = -1; c <= 1; ++c)
            for (int bq = -1; bq <= 1; ++bq) {
                const T wzy = w[c + 1] * w[bq + 1];
                const long o = f + bq * sy + c * sz;
                acc += wzy * (w[0] * rr[o - 1] + w[1] * rr[o] + w[2] * rr[o + 1]);
            }
    } else {
        const long f = 2L * I;
        acc = w[0] * rr[f - 1] + w[1] * rr[f] + w[2] * rr[f + 1];
    }
    fp(bc, q)[cc] = acc;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void resid_restrict_kernel(Tiling t, double alpha, View<T> b, View<T> u,
                                                               View<T> bc)
{
    Pt q; int I, J, K; long cc;
    if (!tile_point<DIM>(t, q, I, J, K, cc)) return;
    const int nf = 2 * (q.n + 1) - 1;
    const T ah = (T)ah_d(q.par(alpha), nf);
    const T *uu = fp(u, q);
    const T *bb = fp(b, q);
    const long sy = row_stride(nf), sz = plane_stride(nf);
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    T acc = 0;
    if (DIM == 3) {
        const long f = 2L * I + 2L * J * sy + 2L * K * sz;
        // one fine plane at a time: its nine residuals' loads issue together
        for (int c = -1; c <= 1; ++c)
#pragma unroll
            for (int bq = -1; bq <= 1; ++bq) {
                const T wzy = w[c + 1] * w[bq + 1];
                T row = 0;
#pragma unroll
                for (int a = -1; a <= 1; ++a) {
                    const long o = f + a + bq * sy + c * sz;
                    const T res = bb[o] - (uu[o] - ah * d2sum<3>(uu, o, sy, sz));
                    row += w[a + 1] * res;
                }
                acc += wzy * row;
            }
    } else {
        const long f = 2L * I;
        for (int a = -1; a <= 1; ++a) {
            const long o = f + a;
            const T res = bb[o] - (uu[o] - ah * d2sum<1>(uu, o, sy, sz));
            acc += w[a + 1] * res;
        }
    }
    fp(bc, q)[cc] = acc;
}

// -------------------------------------------------------- prolongation
// q.n = fine n; coarse n = coarser(q.n).  Coarse halo entries are zero, so
// the boundary needs no special case.
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void prolong_kernel(Tiling t, View<T> ec, View<T> u)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    const int nc = coarser(q.n);
    const T *e = fp(ec, q);
    const long sy = row_stride(nc), sz = plane_stride(nc);
    const int i0 = i >> 1, i1 = (i + 1) >> 1;
    T v;
    if (DIM == 3) {
        const int j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
        auto rowv = [&](int jj, int kk) -> T {
            const long o = jj * sy + kk * sz;
            return (i & 1) ? (T)0.5 * (e[o + i0] + e[o + i1]) : e[o + i0];
        };
        auto planev = [&](int kk) -> T {
            return (j & 1) ? (T)0.5 * (rowv(j0, kk) + rowv(j1, kk)) : rowv(j0, kk);
        };
        v = (k & 1) ? (T)0.5 * (planev(k0) + planev(k1)) : planev(k0);
    } else {
        v = (i & 1) ? (T)0.5 * (e[i0] + e[i1]) : e[i0];
    }
    fp(u, q)[c] += v;
}

// ------------------------------------------------------------ coarsest
// n = 1: one unknown.  n = 2: the eigenvectors of the 2-point Dirichlet
// Laplacian are (1,1) and (1,-1) with eigenvalues -1/h^2 and -3/h^2; in 3D
// their tensor products diagonalise H, so u = sum_s (v_s . b) v_s / (8 lambda_s).
// One thread per field.
template <int DIM, typename T>
__global__ void coarsest_kernel(Tiling t, double alpha, View<T> b, View<T> u)
{
    unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
    Pt q;
    const int *mask;
    if (!find_seg(t, gid, q, mask, [](int) { return 1L; })) return;
    q.item = (int)gid;
    if (mask && !mask[q.item]) return;
    const int n = q.n;
    const T ah = (T)ah_d(q.par(alpha), n);
    const T *bb = fp(b, q);
    T *uu = fp(u, q);
    if (n == 1) {
        const long c = DIM == 3 ? 1 + row_stride(1) + plane_stride(1) : 1;
        uu[c] = bb[c] / ((T)1 + (T)(2 * DIM) * ah);
        return;
    }
    if (DIM == 1) {
        const T b1 = bb[1], b2 = bb[2];
        const T p = (b1 + b2) / ((T)1 + ah), m = (b1 - b2) / ((T)1 + (T)3 * ah);
        uu[1] = (T)0.5 * (p + m);
        uu[2] = (T)0.5 * (p - m);
        return;
    }
    const long sy = row_stride(2), sz = plane_stride(2);
    T bv[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) bv[w] = bb[(w & 1) + 1 + (((w >> 1) & 1) + 1) * sy + ((w >> 2) + 1) * sz];
    T coef[8];
#pragma unroll
    for (int sgn = 0; sgn < 8; ++sgn) {
        T dot = 0;
#pragma unroll
        for (int w = 0; w < 8; ++w) dot += (__builtin_popcount(sgn & w) & 1) ? -bv[w] : bv[w];
        coef[sgn] = dot / ((T)8 * ((T)1 + ah * (T)(3 + 2 * __builtin_popcount(sgn))));
    }
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        T acc = 0;
#pragma unroll
        for (int sgn = 0; sgn < 8; ++sgn) acc += (__builtin_popcount(sgn & w) & 1) ? -coef[sgn] : coef[sgn];
        uu[(w & 1) + 1 + (((w >> 1) & 1) + 1) * sy + ((w >> 2) + 1) * sz] = acc;
    }
}

// ------------------------------------------- column-blocked 3D variants
// Same arithmetic as the point kernels; a thread owns KZ planes of one
// (i, j) column and issues every load before its stores (several KB in
// flight per wavefront; one point per thread leaves HBM latency-bound).
// Loads are not guarded by the column length: a short column (top chunk)
// repeats its last plane, so every load issues at once without branches
// and only the stores are guarded.
constexpr int KZ = 4;

// col[w] = u at plane k0-1+w, w = 0 .. nk+1 (planes 0 and n+1 are halo zeros)
template <typename T>
__device__ inline void load_col(const T *__restrict__ u, long o, long sz, int nk, T (&col)[KZ + 2])
{
#pragma unroll
    for (int w = 0; w < KZ + 2; ++w) col[w] = u[o + (long)(min(w, nk + 1) - 1) * sz];
}

template <typename T>
__device__ inline void load_xy(const T *__restrict__ u, long o, long sy, long sz, int nk, T (&xs)[KZ], T (&ys)[KZ])
{
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        const long c = o + (long)min(w, nk - 1) * sz;
        xs[w] = u[c - 1] + u[c + 1];
        ys[w] = u[c - sy] + u[c + sy];
    }
}

template <typename T>
__device__ inline T d2_of(const T (&col)[KZ + 2], const T (&xs)[KZ], const T (&ys)[KZ], int w)
{
    T s = xs[w];
    s += ys[w] + (col[w] + col[w + 2]);
    return s - (T)6 * col[w + 1];
}

template <typename T, typename TO>
__global__ __launch_bounds__(BLOCK) void resid_kz_kernel(Tiling t, double alpha, View<T> b, View<T> u, View<TO> r)
{
    Pt q; int i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, q, i, j, k0, nk, o)) return;
    const T ah = (T)ah_d(q.par(alpha), q.n);
    const long sy = row_stride(q.n), sz = plane_stride(q.n);
    const T *__restrict__ uu = fp(u, q);
    const T *__restrict__ bb = fp(b, q);
    TO *__restrict__ rr = fp(r, q);
    T col[KZ + 2], xs[KZ], ys[KZ], bv[KZ];
    load_col(uu, o, sz, nk, col);
    load_xy(uu, o, sy, sz, nk, xs, ys);
#pragma unroll
    for (int w = 0; w < KZ; ++w) bv[w] = bb[o + (long)min(w, nk - 1) * sz];
#pragma unroll
    for (int w = 0; w < KZ; ++w)
        if (w < nk) rr[o + (long)w * sz] = (TO)(bv[w] - (col[w + 1] - ah * d2_of(col, xs, ys, w)));
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void jacobi_kz_kernel(Tiling t, double alpha, double omega, View<T> b, View<T> u,
                                                          View<T> out)
{
    Pt q; int i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, q, i, j, k0, nk, o)) return;
    const double a = q.par(alpha);
    const T ah = (T)ah_d(a, q.n), winv = (T)winv_d(a, omega, q.n, 3);
    const long sy = row_stride(q.n), sz = plane_stride(q.n);
    const T *__restrict__ uu = fp(u, q);
    const T *__restrict__ bb = fp(b, q);
    T *__restrict__ oo = fp(out, q);
    T col[KZ + 2], xs[KZ], ys[KZ], bv[KZ];
    load_col(uu, o, sz, nk, col);
    load_xy(uu, o, sy, sz, nk, xs, ys);
#pragma unroll
    for (int w = 0; w < KZ; ++w) bv[w] = bb[o + (long)min(w, nk - 1) * sz];
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        if (w < nk) {
            const T res = bv[w] - (col[w + 1] - ah * d2_of(col, xs, ys, w));
            oo[o + (long)w * sz] = col[w + 1] + winv * res;
        }
    }
}

// u += P ec: the d-linear value at fine (i, j, k) is the z-average of the
// bilinear values of coarse planes k>>1 and (k+1)>>1 (one plane when k even).
// Every load is issued before any arithmetic, without branches around
// them: the four coarse values of each touched plane (the two x and the
// two y neighbours coincide on an even axis; planes past the top are
// clamped to the zero halo plane) and the KZ fine values (repeated from
// the last plane of a short column); the parities pick with selects.
template <typename T>
__global__ __launch_bounds__(BLOCK) void prolong_kz_kernel(Tiling t, View<T> ec, View<T> u)
{
    Pt q; int i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, q, i, j, k0, nk, o)) return;
    const int nc = coarser(q.n);
    const T *__restrict__ e = fp(ec, q);
    T *__restrict__ uu = fp(u, q);
    const int csy = (int)row_stride(nc), csz = (int)plane_stride(nc), sz = (int)plane_stride(q.n);
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1;
    const int c0 = k0 >> 1;                       // first coarse plane touched
    constexpr int NCP = KZ / 2 + 2;               // coarse planes touched by KZ fine planes
    const bool ox = (i & 1) != 0, oy = (j & 1) != 0;
    T c00[NCP], c01[NCP], c10[NCP], c11[NCP], uv[KZ];
#pragma unroll
    for (int cq = 0; cq < NCP; ++cq) {
        const int ob = min(c0 + cq, nc + 1) * csz;
        c00[cq] = e[ob + j0 * csy + i0];
        c01[cq] = e[ob + j0 * csy + i1];
        c10[cq] = e[ob + j1 * csy + i0];
        c11[cq] = e[ob + j1 * csy + i1];
    }
#pragma unroll
    for (int w = 0; w < KZ; ++w) uv[w] = uu[o + (long)min(w, nk - 1) * sz];
    T pv[NCP];
#pragma unroll
    for (int cq = 0; cq < NCP; ++cq) {
        const T r0 = ox ? (T)0.5 * (c00[cq] + c01[cq]) : c00[cq];
        const T r1 = ox ? (T)0.5 * (c10[cq] + c11[cq]) : c10[cq];
        pv[cq] = oy ? (T)0.5 * (r0 + r1) : r0;
    }
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        if (w < nk) {
            const int k = k0 + w;
            const int a = (k >> 1) - c0, bq = ((k + 1) >> 1) - c0;
            const T v = (k & 1) ? (T)0.5 * (pv[a] + pv[bq]) : pv[a];
            uu[o + (long)w * sz] = uv[w] + v;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void copy_kz_kernel(Tiling t, View<T> src, View<T> dst)
{
    Pt q; int i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, q, i, j, k0, nk, o)) return;
    const long sz = plane_stride(q.n);
    const T *__restrict__ a = fp(src, q);
    T *__restrict__ d = fp(dst, q);
    T v[KZ];
#pragma unroll
    for (int w = 0; w < KZ; ++w) v[w] = a[o + (long)min(w, nk - 1) * sz];
#pragma unroll
    for (int w = 0; w < KZ; ++w) if (w < nk) d[o + (long)w * sz] = v[w];
}

__global__ __launch_bounds__(BLOCK) void add_f32_kz_kernel(Tiling t, View<float> e, View<double> u)
{
    Pt q; int i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, q, i, j, k0, nk, o)) return;
    const float *__restrict__ ee = fp(e, q);
    double *__restrict__ uu = fp(u, q);
    const long sz = plane_stride(q.n);
    double uv[KZ];
    float ev[KZ];
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        uv[w] = uu[o + (long)min(w, nk - 1) * sz];
        ev[w] = ee[o + (long)min(w, nk - 1) * sz];
    }
#pragma unroll
    for (int w = 0; w < KZ; ++w) if (w < nk) uu[o + (long)w * sz] = uv[w] + (double)ev[w];
}

// -------------------------------------------------------------- misc
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void zero_kernel(Tiling t, View<T> u)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    fp(u, q)[c] = (T)0;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void copy_kernel(Tiling t, View<T> src, View<T> dst)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    fp(dst, q)[c] = fp(src, q)[c];
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void add_f32_kernel(Tiling t, View<float> e, View<double> u)
{
    Pt q; int i, j, k; long c;
    if (!tile_point<DIM>(t, q, i, j, k, c)) return;
    double *uu = fp(u, q);
    uu[c] = uu[c] + (double)fp(e, q)[c];
}

// Max-reduce non-negative doubles through their bit patterns: for x >= 0
// the IEEE order equals the unsigned order, and NaN (sign cleared) sorts
// above +Inf, so a NaN anywhere survives the reduction.
__device__ inline void block_max_bits(unsigned long long v, unsigned long long *dst)
{
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    __shared__ unsigned long long part[BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = part[0];
        for (int w = 1; w < BLOCK / 64; ++w) m = part[w] > m ? part[w] : m;
        if (m) atomicMax(dst, m);
    }
}

__device__ inline unsigned long long abs_bits(double x) { return (unsigned long long)__double_as_longlong(fabs(x)); }

// Index of field q.item of segment q.sg among all fields of the launch.
__device__ inline int flat_item(const Tiling &t, const Pt &q)
{
    int base = 0;
    for (int s = 0; s < q.sg; ++s) base += t.seg_count(s);
    return base + q.item;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void norm_kernel(Tiling t, View<T> v, unsigned long long *bits)
{
    Pt q; int i, j, k; long c;
    const bool ok = tile_point<DIM>(t, q, i, j, k, c);
    const unsigned long long m = ok ? abs_bits((double)fp(v, q)[c]) : 0ull;
    Pt qb;   // every thread of a workgroup belongs to the same field
    if (!tile_block_item<DIM>(t, qb)) return;
    block_max_bits(m, bits + flat_item(t, qb));
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void resid_norm_kernel(Tiling t, double alpha, View<double> b, View<double> u,
                                                           unsigned long long *bits)
{
    Pt q; int i, j, k; long c;
    const bool ok = tile_point<DIM>(t, q, i, j, k, c);
    unsigned long long m = 0ull;
    if (ok) {
        const double ah = ah_d(q.par(alpha), q.n);
        const double *uu = fp(u, q);
        const double lap = d2sum<DIM>(uu, c, row_stride(q.n), plane_stride(q.n));
        m = abs_bits(fp(b, q)[c] - (uu[c] - ah * lap));
    }
    Pt qb;
    if (!tile_block_item<DIM>(t, qb)) return;
    block_max_bits(m, bits + flat_item(t, qb));
}

// Streaming reference: one 16-byte nontemporal load and store per thread
// and no loop (the shape that copied fastest on gfx950 among unrolled,
// grid-stride and temporal variants).
typedef double dvec2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void stream_copy_kernel(const dvec2 *__restrict__ a, dvec2 *__restrict__ b,
                                                          size_t n16)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, int count)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < count) p[w] = v;
}

inline dim3 grid_of(const Tiling &t) { return dim3((unsigned)grid_blocks(t)); }
inline dim3 col_grid(const Tiling &t) { return dim3((unsigned)col_blocks<KZ>(t)); }

// Same launch on the next-coarser grid of every segment.
inline Tiling coarsen(const Tiling &t)
{
    Tiling c = t;
    c.n = coarser(t.n);
    for (int s = 1; s < t.nseg; ++s) c.x[s - 1].n = coarser(t.x[s - 1].n);
    return c;
}

#define PFMG_DISPATCH(t, KER, ...)                                                          \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                 \
        else KER<1><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                              \
        return hipGetLastError();                                                           \
    } while (0)

#define PFMG_DISPATCH_T(t, KER, T, ...)                                                     \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3, T><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);              \
        else KER<1, T><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                           \
        return hipGetLastError();                                                           \
    } while (0)

}  // namespace

namespace k {

template <typename T>
hipError_t resid(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> r, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) resid_kz_kernel<T, T><<<col_grid(t), BLOCK, 0, s>>>(t, alpha, b, u, r);
    else resid_kernel<1, T, T><<<grid_of(t), BLOCK, 0, s>>>(t, alpha, b, u, r);
    return hipGetLastError();
}

hipError_t resid_round(const Tiling &t, double alpha, View<double> b, View<double> u, View<float> r32,
                       hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) resid_kz_kernel<double, float><<<col_grid(t), BLOCK, 0, s>>>(t, alpha, b, u, r32);
    else resid_kernel<1, double, float><<<grid_of(t), BLOCK, 0, s>>>(t, alpha, b, u, r32);
    return hipGetLastError();
}

template <typename T>
hipError_t jacobi(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, View<T> out, hipStream_t s)
{
    if (stencil_z_ok(t)) return jacobi_z(t, alpha, omega, b, u, out, s);
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) return launch(jacobi_kz_kernel<T>, col_grid(t), dim3(BLOCK), 0, s, t, alpha, omega, b, u, out);
    jacobi_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, alpha, omega, b, u, out);
    return hipGetLastError();
}

template <typename T>
hipError_t jacobi_zero(const Tiling &t, double alpha, double omega, View<T> b, View<T> out, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) return launch(jacobi_zero_kernel<3, T>, grid_of(t), dim3(BLOCK), 0, s, t, alpha, omega, b, out);
    jacobi_zero_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, alpha, omega, b, out);
    return hipGetLastError();
}

template <typename T>
hipError_t rbgs(const Tiling &t, double alpha, double omega, int colour, View<T> b, View<T> u, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) return launch(rbgs_kernel<3, T>, grid_of(t), dim3(BLOCK), 0, s, t, alpha, omega, colour, b, u);
    rbgs_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, alpha, omega, colour, b, u);
    return hipGetLastError();
}

template <typename T>
hipError_t rbgs_zero_red(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) return launch(rbgs_zero_red_kernel<3, T>, grid_of(t), dim3(BLOCK), 0, s, t, alpha, omega, b, u);
    rbgs_zero_red_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, alpha, omega, b, u);
    return hipGetLastError();
}

template <typename T>
hipError_t restrict_fw(const Tiling &t, View<T> r, View<T> bc, hipStream_t s)
{
    const Tiling tc = coarsen(t);
    PFMG_DISPATCH_T(tc, restrict_kernel, T, tc, r, bc);
}

template <typename T>
hipError_t resid_restrict(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> bc, hipStream_t s)
{
    if (resid_restrict_z_ok(t)) return resid_restrict_z(t, alpha, b, u, bc, s);
    const Tiling tc = coarsen(t);
    PFMG_DISPATCH_T(tc, resid_restrict_kernel, T, tc, alpha, b, u, bc);
}

template <typename T>
hipError_t prolong_add(const Tiling &t, View<T> ec, View<T> u, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    // PFMG_PROLONG_Z=0 keeps the column kernel for every launch
    static const bool use_z = [] {
        const char *e = getenv("PFMG_PROLONG_Z");
        return !(e && atoi(e) == 0);
    }();
    if (t.dim == 3 && use_z && prolong_z_ok(t)) return prolong_z(t, ec, u, s);
    if (t.dim == 3) prolong_kz_kernel<T><<<col_grid(t), BLOCK, 0, s>>>(t, ec, u);
    else prolong_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, ec, u);
    return hipGetLastError();
}

template <typename T>
hipError_t coarsest(const Tiling &t, double alpha, View<T> b, View<T> u, hipStream_t s)
{
    long items = 0;
    for (int sg = 0; sg < t.nseg; ++sg) items += t.seg_count(sg);
    if (items == 0) return hipSuccess;
    const unsigned nb = (unsigned)((items + 63) / 64);
    if (t.dim == 3) coarsest_kernel<3, T><<<nb, 64, 0, s>>>(t, alpha, b, u);
    else coarsest_kernel<1, T><<<nb, 64, 0, s>>>(t, alpha, b, u);
    return hipGetLastError();
}

template <typename T>
hipError_t zero(const Tiling &t, View<T> u, hipStream_t s)
{
    PFMG_DISPATCH_T(t, zero_kernel, T, t, u);
}

template <typename T>
hipError_t copy(const Tiling &t, View<T> src, View<T> dst, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) copy_kz_kernel<T><<<col_grid(t), BLOCK, 0, s>>>(t, src, dst);
    else copy_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, src, dst);
    return hipGetLastError();
}

hipError_t add_f32(const Tiling &t, View<float> e, View<double> u, hipStream_t s)
{
    if (t.dim == 3 && grid_blocks(t) > 0) {
        add_f32_kz_kernel<<<col_grid(t), BLOCK, 0, s>>>(t, e, u);
        return hipGetLastError();
    }
    PFMG_DISPATCH(t, add_f32_kernel, t, e, u);
}

template <typename T>
hipError_t norm_inf(const Tiling &t, View<T> v, unsigned long long *bits, hipStream_t s)
{
    PFMG_DISPATCH_T(t, norm_kernel, T, t, v, bits);
}

hipError_t resid_norm(const Tiling &t, double alpha, View<double> b, View<double> u, unsigned long long *bits,
                      hipStream_t s)
{
    PFMG_DISPATCH(t, resid_norm_kernel, t, alpha, b, u, bits);
}

hipError_t stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks > 0xffffffffull) return hipErrorInvalidValue;
    stream_copy_kernel<<<(unsigned)blocks, 256, 0, s>>>((const dvec2 *)src, (dvec2 *)dst, n16);
    return hipGetLastError();
}

hipError_t fill_u64(unsigned long long *p, unsigned long long v, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    fill_u64_kernel<<<(count + 255) / 256, 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}

#define PFMG_INST(T)                                                                                         \
    template hipError_t resid<T>(const Tiling &, double, View<T>, View<T>, View<T>, hipStream_t);            \
    template hipError_t jacobi<T>(const Tiling &, double, double, View<T>, View<T>, View<T>, hipStream_t);   \
    template hipError_t jacobi_zero<T>(const Tiling &, double, double, View<T>, View<T>, hipStream_t);       \
    template hipError_t rbgs<T>(const Tiling &, double, double, int, View<T>, View<T>, hipStream_t);         \
    template hipError_t rbgs_zero_red<T>(const Tiling &, double, double, View<T>, View<T>, hipStream_t);     \
    template hipError_t restrict_fw<T>(const Tiling &, View<T>, View<T>, hipStream_t);                       \
    template hipError_t resid_restrict<T>(const Tiling &, double, View<T>, View<T>, View<T>, hipStream_t);   \
    template hipError_t prolong_add<T>(const Tiling &, View<T>, View<T>, hipStream_t);                       \
    template hipError_t coarsest<T>(const Tiling &, double, View<T>, View<T>, hipStream_t);                  \
    template hipError_t zero<T>(const Tiling &, View<T>, hipStream_t);                                       \
    template hipError_t copy<T>(const Tiling &, View<T>, View<T>, hipStream_t);                              \
    template hipError_t norm_inf<T>(const Tiling &, View<T>, unsigned long long *, hipStream_t);

PFMG_INST(double)
PFMG_INST(float)

}  // namespace k
}  // namespace pfmg
