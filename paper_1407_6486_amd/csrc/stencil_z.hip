// Out-of-place 7-point stencils in one z-marching pass (3D, 31 <= n <= 255):
//   F = c L_h u: the F = nu L_h U of every node after its solve and after
//     the spatial interpolation of PFASST (Sec. 2.4), 16 bytes per point;
//   u' = u + w (b - (u - ah L u)): one omega-Jacobi sweep of the V-cycle
//     (Sec. 4.1.1, w = omega / (1 + 6 ah), ah = alpha (n+1)^2), 24 bytes
//     per point.
//
// A workgroup owns full x-rows, TY output rows and a chunk of z planes and
// marches through it in z (upwards in even chunks, downwards in odd ones, so
// that neighbouring chunks read their shared border planes at about the same
// time and the second read hits the XCD's L2).  At step k the rows
// j0-1 .. j0+TY of plane k go into one of four LDS buffers and the output is
// computed on the plane before k from the x and y neighbours in LDS and the
// z neighbours in registers; u is read
// once (plus the halo rows that neighbouring tiles also read) and the output
// written once.  The loads of step k + 1 are issued before step k's
// arithmetic.  The arithmetic per point is that of the column-blocked
// kernels they replace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace pfmg {
namespace {

constexpr int TY = 4;   // output rows per workgroup

// RLN: x lanes per row; Q = ceil((TY + 2) / (BLOCK / RLN)) rows per thread.
// JAC: Jacobi sweep (b read, c = alpha, omega given) instead of F = c L u.
//
// The march has no divergent branches around its loads: a thread's rows
// are wave-uniform, loads read clamped indices (zero halo words outside the
// interior), the u planes sit in register slots and LDS buffers indexed by
// the plane modulo 4 and the loop is unrolled four times; every step first
// waits for the loads of the previous step, then issues its own.
template <typename T, int RLN, int Q, bool JAC>
__global__ __launch_bounds__(BLOCK) void stencil_z_kernel(Tiling t, int zchunk, double c, double omega, View<T> b,
                                                          View<T> u, View<T> F)
{
    constexpr int RL = RLN + 2;
    constexpr int RPP = BLOCK / RLN;
    constexpr int ROWS = TY + 2;             // rows j0-1 .. j0+TY
    static_assert(Q * RPP >= ROWS, "rows per thread");
    extern __shared__ unsigned char smem_raw[];
    T *lp = reinterpret_cast<T *>(smem_raw);             // 4 planes of ROWS rows

    unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [zchunk](int nn) {
            return (long)((nn + TY - 1) / TY) * ((nn + zchunk - 1) / zchunk);
        }))
        return;
    const int n = qs.n;
    const int ytiles = (n + TY - 1) / TY, zch = (n + zchunk - 1) / zchunk;
    const int item = (int)(bid / (unsigned)(ytiles * zch));
    const int rem = (int)(bid - (unsigned)item * (unsigned)(ytiles * zch));
    const int jt = rem / zch, zc = rem - jt * zch;
    if (mask && !mask[item]) return;
    qs.item = item;
    const double cc = qs.par(c), ih2 = (double)(n + 1) * (double)(n + 1);
    const double ahd = cc * (double)(n + 1) * (double)(n + 1);
    const T ah = (T)ahd, winv = (T)(omega / (1.0 + 2.0 * 3 * ahd));
    const int j0 = jt * TY + 1, k0 = zc * zchunk + 1;
    const int k1 = min(k0 + zchunk, n + 1);  // F on planes k0 .. k1-1
    // step v = 0 .. V works on plane kv(v) and writes plane kv(v - 1); the
    // z-neighbour sums commute, so both directions give the same numbers
    const int dk = (zc & 1) ? -1 : 1, V = k1 - k0 + 1;
    auto kv = [&](int v) { return dk > 0 ? k0 - 1 + v : k1 - v; };
    const int i = (int)(threadIdx.x % RLN) + 1;
    const int rsub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / RLN));
    const bool xin = i <= n;
    // element offsets inside one field fit in 32 bits (n <= 255)
    const int sy = (int)row_stride(n), sz = (int)plane_stride(n);
    const T *__restrict__ U = fp(u, qs);
    const T *__restrict__ Bv = JAC ? fp(b, qs) : nullptr;
    T *__restrict__ Fo = fp(F, qs);
    // lanes past the row read its right halo word (zero)
    const unsigned ib = (unsigned)min(i, n + 1) * (unsigned)sizeof(T);

    for (int r = threadIdx.x; r < 4 * ROWS; r += BLOCK) lp[r * RL] = (T)0;

    // per row (uniform): ownership, clamped byte offset
    bool own[Q];
    unsigned roff[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = rsub + q * RPP, j = j0 - 1 + r;
        own[q] = r < ROWS;
        roff[q] = (unsigned)(min(max(j, 0), n + 1) * sy) * (unsigned)sizeof(T);
    }
    auto planeb = [&](int k) { return (unsigned)(min(max(k, 0), n + 1) * sz) * (unsigned)sizeof(T); };
    auto ld = [&](const T *__restrict__ a, unsigned rb, unsigned pb) -> T {
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(a) + (rb + pb) + ib);
    };

    // the u plane of step v in slot v & 3, its b plane in v & 1
    T us[4][Q], bs[2][Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        us[0][q] = us[1][q] = us[2][q] = us[3][q] = (T)0;
        bs[0][q] = bs[1][q] = (T)0;
    }
    {
        const unsigned p0 = planeb(kv(0));
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (own[q]) us[0][q] = ld(U, roff[q], p0);
    }

    // step v on plane k = kv(v) (slot S): u plane k to LDS, output on the
    // plane before it
    auto step = [&](auto sc, int v) {
        constexpr int S = decltype(sc)::value;
        const int k = kv(v);
        constexpr int S1 = (S + 1) & 3, S2 = (S + 2) & 3, S3 = (S + 3) & 3;
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the previous step's loads
        __builtin_amdgcn_sched_barrier(0);
        if (v < V) {
            const unsigned pu = planeb(k + dk), pb = planeb(k);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int r = rsub + q * RPP;
                if (own[q]) us[S1][q] = ld(U, roff[q], pu);
                if (JAC && r >= 1 && r <= TY) bs[S & 1][q] = ld(Bv, roff[q], pb);
            }
        }
        // ---- u plane k -> LDS (4 buffers: plane k-1's buffer is not
        // rewritten before every thread has passed the next barrier)
        T *buf = lp + S * ROWS * RL;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * RPP;
            if (own[q]) buf[r * RL + i] = us[S][q];
        }
        __syncthreads();
        // ---- output on plane kb, the previous step's
        const int kb = k - dk;
        if (kb >= k0 && kb < k1 && xin) {
            const T *bb = lp + S3 * ROWS * RL;
            const int ko = kb * sz;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int r = rsub + q * RPP, j = j0 - 1 + r;
                if (r >= 1 && r <= TY && j <= n) {
                    const T *row = bb + r * RL;
                    T s = row[i - 1] + row[i + 1];
                    s += (bb[(r - 1) * RL + i] + bb[(r + 1) * RL + i]) + (us[S2][q] + us[S][q]);
                    s -= (T)6 * us[S3][q];
                    if (JAC) {
                        const T res = bs[(S + 1) & 1][q] - (us[S3][q] - ah * s);
                        Fo[i + j * sy + ko] = us[S3][q] + winv * res;
                    } else {
                        Fo[i + j * sy + ko] = (T)(cc * (ih2 * (double)s));
                    }
                }
            }
        }
    };
    for (int vv = 0; vv <= V; vv += 4) {
        step(std::integral_constant<int, 0>{}, vv);
        if (vv + 1 > V) break;
        step(std::integral_constant<int, 1>{}, vv + 1);
        if (vv + 2 > V) break;
        step(std::integral_constant<int, 2>{}, vv + 2);
        if (vv + 3 > V) break;
        step(std::integral_constant<int, 3>{}, vv + 3);
    }
}

}  // namespace

namespace k {

// Small launches (a single 63^3 field of the coarse chain) take the
// column-blocked kernel: with few workgroups the z march is latency-bound.
bool stencil_z_ok(const Tiling &t)
{
    if (t.dim != 3) return false;
    long points = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        if (t.seg_count(sg) > 0 && (t.seg_n(sg) < 31 || t.seg_n(sg) > 255)) return false;
        points += (long)t.seg_count(sg) * t.seg_n(sg) * t.seg_n(sg) * t.seg_n(sg);
    }
    return points >= (1L << 20);
}

template <typename T, bool JAC>
hipError_t stencil_z(const Tiling &t, double c, double omega, View<T> b, View<T> u, View<T> F, hipStream_t s)
{
    if (!stencil_z_ok(t)) return hipErrorInvalidValue;
    int nmax = 0;
    long rows_total = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        nmax = std::max(nmax, t.seg_n(sg));
        rows_total += (long)t.seg_count(sg) * ((t.seg_n(sg) + TY - 1) / TY);
    }
    if (rows_total == 0) return hipSuccess;
    // z chunks: about 1024 workgroups in all, at least 4 planes each, and at
    // least two chunks (with one, a launch of many fields, e.g. 60 x 127^3,
    // ran 1920 whole-height marches, a quarter of them in a second, mostly
    // empty round: 496 against 464 us with two)
    const long chunks = std::min<long>(std::max(1, nmax / 4), std::max<long>(2, (1024 + rows_total - 1) / rows_total));
    const int zchunk = (int)((nmax + chunks - 1) / chunks);
    long blocks = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        const int n = t.seg_n(sg);
        blocks += (long)t.seg_count(sg) * ((n + TY - 1) / TY) * ((n + zchunk - 1) / zchunk);
    }
    const int rln = nmax <= 64 ? 64 : nmax <= 128 ? 128 : 256;
    const size_t lds = (size_t)4 * (TY + 2) * (rln + 2) * sizeof(T);
    const dim3 g((unsigned)blocks), blk(BLOCK);
    if (rln == 64) return launch(stencil_z_kernel<T, 64, 2, JAC>, g, blk, lds, s, t, zchunk, c, omega, b, u, F);
    if (rln == 128) return launch(stencil_z_kernel<T, 128, 3, JAC>, g, blk, lds, s, t, zchunk, c, omega, b, u, F);
    return launch(stencil_z_kernel<T, 256, 6, JAC>, g, blk, lds, s, t, zchunk, c, omega, b, u, F);
}

hipError_t apply_L_z(const Tiling &t, double c, View<double> u, View<double> F, hipStream_t s)
{
    return stencil_z<double, false>(t, c, 0.0, View<double>{nullptr, 0}, u, F, s);
}

template <typename T>
hipError_t jacobi_z(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, View<T> out, hipStream_t s)
{
    return stencil_z<T, true>(t, alpha, omega, b, u, out, s);
}

template hipError_t jacobi_z<double>(const Tiling &, double, double, View<double>, View<double>, View<double>,
                                     hipStream_t);
template hipError_t jacobi_z<float>(const Tiling &, double, double, View<float>, View<float>, View<float>,
                                    hipStream_t);

}  // namespace k
}  // namespace pfmg
