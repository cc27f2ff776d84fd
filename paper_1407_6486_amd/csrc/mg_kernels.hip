// Geometric multigrid kernels for (I - alpha L_h) u = b on gfx950.
//
// The node solves of the SDC sweep (eq. SDCcompactLIII, alpha = nu dt_m)
// are done with V-cycles: pre/post smoothing, residual, full-weighting
// restriction, linear interpolation (Sec. 4.1.1, Sec. 4.2.1).  Coarse
// operators are re-discretised on h_{l+1} = 2 h_l with the same alpha;
// grids with n in {1, 2} are solved exactly.
//
// All kernels are memory-bound stencils: one thread per point, whole
// 64-point row segments per wavefront, no matrix cores.  FP64 and FP32
// instances serve the plain and the mixed-precision forms.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace pfmg {
namespace {

template <typename T>
__device__ inline T *fp(View<T> v, int item) { return v.p + (long)item * v.stride; }

// ---------------------------------------------------------------- residual
template <int DIM, typename T, typename TO>
__global__ __launch_bounds__(BLOCK) void resid_kernel(Tiling t, T ah, View<T> b, View<T> u, View<TO> r)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    const T *uu = fp(u, item);
    const long sy = row_stride(t.n), sz = plane_stride(t.n);
    const T lap = d2sum<DIM>(uu, c, sy, sz);
    fp(r, item)[c] = (TO)(fp(b, item)[c] - (uu[c] - ah * lap));
}

// ------------------------------------------------------------------ Jacobi
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void jacobi_kernel(Tiling t, T ah, T winv, View<T> b, View<T> u, View<T> out)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    const T *uu = fp(u, item);
    const long sy = row_stride(t.n), sz = plane_stride(t.n);
    const T lap = d2sum<DIM>(uu, c, sy, sz);
    const T res = fp(b, item)[c] - (uu[c] - ah * lap);
    fp(out, item)[c] = uu[c] + winv * res;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void jacobi_zero_kernel(Tiling t, T winv, View<T> b, View<T> out)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    fp(out, item)[c] = winv * fp(b, item)[c];
}

// --------------------------------------------------------------- red-black
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void rbgs_kernel(Tiling t, T ah, T winv, int colour, View<T> b, View<T> u)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    const int par = (DIM == 3 ? (i + j + k) : i) & 1;
    if (par != colour) return;
    T *uu = fp(u, item);
    const long sy = row_stride(t.n), sz = plane_stride(t.n);
    const T lap = d2sum<DIM>(uu, c, sy, sz);
    const T res = fp(b, item)[c] - (uu[c] - ah * lap);
    uu[c] = uu[c] + winv * res;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void rbgs_zero_red_kernel(Tiling t, T winv, View<T> b, View<T> u)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    const int par = (DIM == 3 ? (i + j + k) : i) & 1;
    fp(u, item)[c] = par == 0 ? winv * fp(b, item)[c] : (T)0;
}

// -------------------------------------------------------------- restriction
// t.n is the coarse n here; nf the fine n.
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void restrict_kernel(Tiling t, int nf, View<T> r, View<T> bc)
{
    int item, I, J, K; long cc;
    if (!tile_point<DIM>(t, item, I, J, K, cc)) return;
    const T *rr = fp(r, item);
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
    fp(bc, item)[cc] = acc;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void resid_restrict_kernel(Tiling t, int nf, T ah, View<T> b, View<T> u, View<T> bc)
{
    int item, I, J, K; long cc;
    if (!tile_point<DIM>(t, item, I, J, K, cc)) return;
    const T *uu = fp(u, item);
    const T *bb = fp(b, item);
    const long sy = row_stride(nf), sz = plane_stride(nf);
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    T acc = 0;
    if (DIM == 3) {
        const long f = 2L * I + 2L * J * sy + 2L * K * sz;
        for (int c = -1; c <= 1; ++c)
            for (int bq = -1; bq <= 1; ++bq) {
                const T wzy = w[c + 1] * w[bq + 1];
                T row = 0;
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
    fp(bc, item)[cc] = acc;
}

// ------------------------------------------------------------ prolongation
// t.n = fine n; coarse n = coarser(t.n).  Coarse halo entries are zero, so
// the boundary needs no special case.
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void prolong_kernel(Tiling t, View<T> ec, View<T> u)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    const int nc = coarser(t.n);
    const T *e = fp(ec, item);
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
    fp(u, item)[c] += v;
}

// --------------------------------------------------------------- coarsest
// n = 1: one unknown.  n = 2: the eigenvectors of the 2-point Dirichlet
// Laplacian are (1,1) and (1,-1) with eigenvalues -1/h^2 and -3/h^2; in 3D
// their tensor products diagonalise H, so u = sum_s (v_s . b) v_s / (8 lambda_s).
template <int DIM, typename T>
__global__ void coarsest_kernel(int n, int count, const int *mask, T ah, View<T> b, View<T> u)
{
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= count || (mask && !mask[item])) return;
    const T *bb = fp(b, item);
    T *uu = fp(u, item);
    if (n == 1) {
        const long c = DIM == 3 ? 1 + row_stride(1) + plane_stride(1) : 1;
        uu[c] = bb[c] / ((T)1 + (T)(2 * DIM) * ah);
        return;
    }
    // n == 2
    if (DIM == 1) {
        const T b1 = bb[1], b2 = bb[2];
        const T p = (b1 + b2) / ((T)1 + ah), q = (b1 - b2) / ((T)1 + (T)3 * ah);
        uu[1] = (T)0.5 * (p + q);
        uu[2] = (T)0.5 * (p - q);
        return;
    }
    const long sy = row_stride(2), sz = plane_stride(2);
    T bv[8];
    for (int q = 0; q < 8; ++q) {
        const int ii = (q & 1) + 1, jj = ((q >> 1) & 1) + 1, kk = (q >> 2) + 1;
        bv[q] = bb[ii + jj * sy + kk * sz];
    }
    T coef[8];
    for (int s = 0; s < 8; ++s) {
        T dot = 0;
        for (int q = 0; q < 8; ++q) {
            int sign = 1;
            for (int d = 0; d < 3; ++d)
                if (((s >> d) & 1) && ((q >> d) & 1)) sign = -sign;
            dot += sign > 0 ? bv[q] : -bv[q];
        }
        const int nneg = (s & 1) + ((s >> 1) & 1) + ((s >> 2) & 1);
        const T lam = (T)1 + ah * (T)(3 + 2 * nneg);   // sum_d (1 or 3)
        coef[s] = dot / ((T)8 * lam);
    }
    for (int q = 0; q < 8; ++q) {
        T acc = 0;
        for (int s = 0; s < 8; ++s) {
            int sign = 1;
            for (int d = 0; d < 3; ++d)
                if (((s >> d) & 1) && ((q >> d) & 1)) sign = -sign;
            acc += sign > 0 ? coef[s] : -coef[s];
        }
        const int ii = (q & 1) + 1, jj = ((q >> 1) & 1) + 1, kk = (q >> 2) + 1;
        uu[ii + jj * sy + kk * sz] = acc;
    }
}

// ------------------------------------------- column-blocked 3D variants
// Same arithmetic as the point kernels above; a thread owns KZ planes of one
// (i, j) column (tile_col) and issues every load before its stores.
constexpr int KZ = 4;

// col[q] = u at plane k0-1+q, q = 0 .. nk+1 (planes 0 and n+1 are halo zeros)
template <typename T>
__device__ inline void load_col(const T *__restrict__ u, long o, long sz, int nk, T (&col)[KZ + 2])
{
#pragma unroll
    for (int q = 0; q < KZ + 2; ++q) col[q] = q <= nk + 1 ? u[o + (long)(q - 1) * sz] : (T)0;
}

template <typename T>
__device__ inline void load_xy(const T *__restrict__ u, long o, long sy, long sz, int nk, T (&xs)[KZ], T (&ys)[KZ])
{
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        if (q < nk) {
            const long c = o + (long)q * sz;
            xs[q] = u[c - 1] + u[c + 1];
            ys[q] = u[c - sy] + u[c + sy];
        }
    }
}

template <typename T>
__device__ inline T d2_of(const T (&col)[KZ + 2], const T (&xs)[KZ], const T (&ys)[KZ], int q)
{
    T s = xs[q];
    s += ys[q] + (col[q] + col[q + 2]);
    return s - (T)6 * col[q + 1];
}

template <typename T, typename TO>
__global__ __launch_bounds__(BLOCK) void resid_kz_kernel(Tiling t, T ah, View<T> b, View<T> u, View<TO> r)
{
    int item, i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, item, i, j, k0, nk, o)) return;
    const long sy = row_stride(t.n), sz = plane_stride(t.n);
    const T *__restrict__ uu = fp(u, item);
    const T *__restrict__ bb = fp(b, item);
    TO *__restrict__ rr = fp(r, item);
    T col[KZ + 2], xs[KZ], ys[KZ], bv[KZ];
    load_col(uu, o, sz, nk, col);
    load_xy(uu, o, sy, sz, nk, xs, ys);
#pragma unroll
    for (int q = 0; q < KZ; ++q) if (q < nk) bv[q] = bb[o + (long)q * sz];
#pragma unroll
    for (int q = 0; q < KZ; ++q)
        if (q < nk) rr[o + (long)q * sz] = (TO)(bv[q] - (col[q + 1] - ah * d2_of(col, xs, ys, q)));
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void jacobi_kz_kernel(Tiling t, T ah, T winv, View<T> b, View<T> u, View<T> out)
{
    int item, i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, item, i, j, k0, nk, o)) return;
    const long sy = row_stride(t.n), sz = plane_stride(t.n);
    const T *__restrict__ uu = fp(u, item);
    const T *__restrict__ bb = fp(b, item);
    T *__restrict__ oo = fp(out, item);
    T col[KZ + 2], xs[KZ], ys[KZ], bv[KZ];
    load_col(uu, o, sz, nk, col);
    load_xy(uu, o, sy, sz, nk, xs, ys);
#pragma unroll
    for (int q = 0; q < KZ; ++q) if (q < nk) bv[q] = bb[o + (long)q * sz];
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        if (q < nk) {
            const T res = bv[q] - (col[q + 1] - ah * d2_of(col, xs, ys, q));
            oo[o + (long)q * sz] = col[q + 1] + winv * res;
        }
    }
}

// u += P ec: the d-linear value at fine (i, j, k) is the z-average of the
// bilinear values of coarse planes k>>1 and (k+1)>>1 (one plane when k even).
template <typename T>
__global__ __launch_bounds__(BLOCK) void prolong_kz_kernel(Tiling t, View<T> ec, View<T> u)
{
    int item, i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, item, i, j, k0, nk, o)) return;
    const int nc = coarser(t.n);
    const T *__restrict__ e = fp(ec, item);
    T *__restrict__ uu = fp(u, item);
    const long csy = row_stride(nc), csz = plane_stride(nc), sz = plane_stride(t.n);
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1;
    const int c0 = k0 >> 1;                       // first coarse plane touched
    constexpr int NCP = KZ / 2 + 2;               // coarse planes touched by KZ fine planes
    T pv[NCP], uv[KZ];
#pragma unroll
    for (int cq = 0; cq < NCP; ++cq) {
        const int kk = c0 + cq;
        T v = (T)0;
        if (kk <= nc + 1) {
            const long ob = (long)kk * csz;
            auto rowv = [&](int jj) -> T {
                const long orow = ob + (long)jj * csy;
                return (i & 1) ? (T)0.5 * (e[orow + i0] + e[orow + i1]) : e[orow + i0];
            };
            v = (j & 1) ? (T)0.5 * (rowv(j0) + rowv(j1)) : rowv(j0);
        }
        pv[cq] = v;
    }
#pragma unroll
    for (int q = 0; q < KZ; ++q) if (q < nk) uv[q] = uu[o + (long)q * sz];
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        if (q < nk) {
            const int k = k0 + q;
            const int a = (k >> 1) - c0, bq = ((k + 1) >> 1) - c0;
            const T v = (k & 1) ? (T)0.5 * (pv[a] + pv[bq]) : pv[a];
            uu[o + (long)q * sz] = uv[q] + v;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void copy_kz_kernel(Tiling t, View<T> src, View<T> dst)
{
    int item, i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, item, i, j, k0, nk, o)) return;
    const long sz = plane_stride(t.n);
    const T *__restrict__ a = fp(src, item);
    T *__restrict__ d = fp(dst, item);
    T v[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) if (q < nk) v[q] = a[o + (long)q * sz];
#pragma unroll
    for (int q = 0; q < KZ; ++q) if (q < nk) d[o + (long)q * sz] = v[q];
}

__global__ __launch_bounds__(BLOCK) void add_f32_kz_kernel(Tiling t, View<float> e, View<double> u)
{
    int item, i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, item, i, j, k0, nk, o)) return;
    const float *__restrict__ ee = fp(e, item);
    double *__restrict__ uu = fp(u, item);
    const long sz = plane_stride(t.n), ez = plane_stride(t.n);
    double uv[KZ];
    float ev[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        if (q < nk) {
            uv[q] = uu[o + (long)q * sz];
            ev[q] = ee[o + (long)q * ez];
        }
    }
#pragma unroll
    for (int q = 0; q < KZ; ++q) if (q < nk) uu[o + (long)q * sz] = uv[q] + (double)ev[q];
}

inline dim3 col_grid(const Tiling &t) { return dim3((unsigned)(col_tiles_per_field(t.n, KZ) * t.count)); }

// ------------------------------------------------------------------- misc
template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void zero_kernel(Tiling t, View<T> u)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    fp(u, item)[c] = (T)0;
}

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void copy_kernel(Tiling t, View<T> src, View<T> dst)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    fp(dst, item)[c] = fp(src, item)[c];
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void add_f32_kernel(Tiling t, View<float> e, View<double> u)
{
    int item, i, j, k; long c;
    if (!tile_point<DIM>(t, item, i, j, k, c)) return;
    double *uu = fp(u, item);
    uu[c] = uu[c] + (double)fp(e, item)[c];
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
        for (int q = 1; q < BLOCK / 64; ++q) m = part[q] > m ? part[q] : m;
        if (m) atomicMax(dst, m);
    }
}

__device__ inline unsigned long long abs_bits(double x) { return (unsigned long long)__double_as_longlong(fabs(x)); }

template <int DIM, typename T>
__global__ __launch_bounds__(BLOCK) void norm_kernel(Tiling t, View<T> v, unsigned long long *bits)
{
    int item, i, j, k; long c;
    const bool ok = tile_point<DIM>(t, item, i, j, k, c);
    unsigned long long m = ok ? abs_bits((double)fp(v, item)[c]) : 0ull;
    // every thread of a block belongs to the same item
    const unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    const int blk_item = (int)(bid / tiles_per_field(t.n, DIM));
    if (blk_item >= t.count) return;
    block_max_bits(m, bits + blk_item);
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void resid_norm_kernel(Tiling t, double ah, View<double> b, View<double> u,
                                                           unsigned long long *bits)
{
    int item, i, j, k; long c;
    const bool ok = tile_point<DIM>(t, item, i, j, k, c);
    unsigned long long m = 0ull;
    if (ok) {
        const double *uu = fp(u, item);
        const double lap = d2sum<DIM>(uu, c, row_stride(t.n), plane_stride(t.n));
        m = abs_bits(fp(b, item)[c] - (uu[c] - ah * lap));
    }
    const unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    const int blk_item = (int)(bid / tiles_per_field(t.n, DIM));
    if (blk_item >= t.count) return;
    block_max_bits(m, bits + blk_item);
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, int count)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) p[q] = v;
}

inline double ah_of(double alpha, int n) { return alpha * (double)(n + 1) * (double)(n + 1); }
inline double winv_of(double alpha, double omega, int n, int dim)
{
    return omega / (1.0 + 2.0 * dim * ah_of(alpha, n));
}

inline dim3 grid_of(const Tiling &t) { return dim3((unsigned)grid_blocks(t)); }

#define PFMG_DISPATCH(t, KER, ...)                                                          \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                 \
        else KER<1><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                              \
        return hipGetLastError();                                                           \
    } while (0)

}  // namespace

namespace k {

template <typename T>
hipError_t resid(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> r, hipStream_t s)
{
    const T ah = (T)ah_of(alpha, t.n);
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) resid_kz_kernel<T, T><<<col_grid(t), BLOCK, 0, s>>>(t, ah, b, u, r);
    else resid_kernel<1, T, T><<<grid_of(t), BLOCK, 0, s>>>(t, ah, b, u, r);
    return hipGetLastError();
}

hipError_t resid_round(const Tiling &t, double alpha, View<double> b, View<double> u, View<float> r32,
                       hipStream_t s)
{
    const double ah = ah_of(alpha, t.n);
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) resid_kz_kernel<double, float><<<col_grid(t), BLOCK, 0, s>>>(t, ah, b, u, r32);
    else resid_kernel<1, double, float><<<grid_of(t), BLOCK, 0, s>>>(t, ah, b, u, r32);
    return hipGetLastError();
}

template <typename T>
hipError_t jacobi(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, View<T> out,
                  hipStream_t s)
{
    const T ah = (T)ah_of(alpha, t.n), wi = (T)winv_of(alpha, omega, t.n, t.dim);
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) jacobi_kz_kernel<T><<<col_grid(t), BLOCK, 0, s>>>(t, ah, wi, b, u, out);
    else jacobi_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, ah, wi, b, u, out);
    return hipGetLastError();
}

template <typename T>
hipError_t jacobi_zero(const Tiling &t, double alpha, double omega, View<T> b, View<T> out, hipStream_t s)
{
    const T wi = (T)winv_of(alpha, omega, t.n, t.dim);
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) jacobi_zero_kernel<3, T><<<grid_of(t), BLOCK, 0, s>>>(t, wi, b, out);
    else jacobi_zero_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, wi, b, out);
    return hipGetLastError();
}

template <typename T>
hipError_t rbgs(const Tiling &t, double alpha, double omega, int colour, View<T> b, View<T> u, hipStream_t s)
{
    const T ah = (T)ah_of(alpha, t.n), wi = (T)winv_of(alpha, omega, t.n, t.dim);
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) rbgs_kernel<3, T><<<grid_of(t), BLOCK, 0, s>>>(t, ah, wi, colour, b, u);
    else rbgs_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, ah, wi, colour, b, u);
    return hipGetLastError();
}

template <typename T>
hipError_t rbgs_zero_red(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, hipStream_t s)
{
    const T wi = (T)winv_of(alpha, omega, t.n, t.dim);
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) rbgs_zero_red_kernel<3, T><<<grid_of(t), BLOCK, 0, s>>>(t, wi, b, u);
    else rbgs_zero_red_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, wi, b, u);
    return hipGetLastError();
}

template <typename T>
hipError_t restrict_fw(const Tiling &t, View<T> r, View<T> bc, hipStream_t s)
{
    Tiling tc = t;
    tc.n = coarser(t.n);
    if (grid_blocks(tc) == 0) return hipSuccess;
    if (t.dim == 3) restrict_kernel<3, T><<<grid_of(tc), BLOCK, 0, s>>>(tc, t.n, r, bc);
    else restrict_kernel<1, T><<<grid_of(tc), BLOCK, 0, s>>>(tc, t.n, r, bc);
    return hipGetLastError();
}

template <typename T>
hipError_t resid_restrict(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> bc, hipStream_t s)
{
    Tiling tc = t;
    tc.n = coarser(t.n);
    const T ah = (T)ah_of(alpha, t.n);
    if (grid_blocks(tc) == 0) return hipSuccess;
    if (t.dim == 3) resid_restrict_kernel<3, T><<<grid_of(tc), BLOCK, 0, s>>>(tc, t.n, ah, b, u, bc);
    else resid_restrict_kernel<1, T><<<grid_of(tc), BLOCK, 0, s>>>(tc, t.n, ah, b, u, bc);
    return hipGetLastError();
}

template <typename T>
hipError_t prolong_add(const Tiling &t, View<T> ec, View<T> u, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) prolong_kz_kernel<T><<<col_grid(t), BLOCK, 0, s>>>(t, ec, u);
    else prolong_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, ec, u);
    return hipGetLastError();
}

template <typename T>
hipError_t coarsest(const Tiling &t, double alpha, View<T> b, View<T> u, hipStream_t s)
{
    const T ah = (T)ah_of(alpha, t.n);
    if (t.count == 0) return hipSuccess;
    const unsigned nb = (t.count + 63) / 64;
    if (t.dim == 3) coarsest_kernel<3, T><<<nb, 64, 0, s>>>(t.n, t.count, t.mask, ah, b, u);
    else coarsest_kernel<1, T><<<nb, 64, 0, s>>>(t.n, t.count, t.mask, ah, b, u);
    return hipGetLastError();
}

template <typename T>
hipError_t zero(const Tiling &t, View<T> u, hipStream_t s)
{
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) zero_kernel<3, T><<<grid_of(t), BLOCK, 0, s>>>(t, u);
    else zero_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, u);
    return hipGetLastError();
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
    if (grid_blocks(t) == 0) return hipSuccess;
    if (t.dim == 3) norm_kernel<3, T><<<grid_of(t), BLOCK, 0, s>>>(t, v, bits);
    else norm_kernel<1, T><<<grid_of(t), BLOCK, 0, s>>>(t, v, bits);
    return hipGetLastError();
}

hipError_t resid_norm(const Tiling &t, double alpha, View<double> b, View<double> u,
                      unsigned long long *bits, hipStream_t s)
{
    const double ah = ah_of(alpha, t.n);
    PFMG_DISPATCH(t, resid_norm_kernel, t, ah, b, u, bits);
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
