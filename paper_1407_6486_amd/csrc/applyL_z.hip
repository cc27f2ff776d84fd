// F = c L_h u in one z-marching pass (3D, 31 <= n <= 255): the F = nu L_h U
// of every node after its solve and after the spatial interpolation of
// PFASST (Sec. 2.4).
//
// A workgroup owns full x-rows, TY output rows and a chunk of z planes and
// marches upwards in z.  At step k the rows j0-1 .. j0+TY of plane k go into
// one of three LDS buffers and F is computed on plane k-1 from the x and y
// neighbours in LDS and the z neighbours in registers; u is read once (plus
// the halo rows that neighbouring tiles also read) and F written once:
// 16 bytes per point in FP64.  The loads of step k + 1 are issued before
// step k's arithmetic.  The arithmetic per point is that of the
// column-blocked kernel it replaces.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace pfmg {
namespace {

constexpr int TY = 4;   // output rows per workgroup

// RLN: x lanes per row; Q = ceil((TY + 2) / (BLOCK / RLN)) rows per thread.
template <int RLN, int Q>
__global__ __launch_bounds__(BLOCK) void apply_L_z_kernel(Tiling t, int zchunk, double c, View<double> u,
                                                          View<double> F)
{
    constexpr int RL = RLN + 2;
    constexpr int RPP = BLOCK / RLN;
    constexpr int ROWS = TY + 2;             // rows j0-1 .. j0+TY
    static_assert(Q * RPP >= ROWS, "rows per thread");
    extern __shared__ unsigned char smem_raw[];
    double *lp = reinterpret_cast<double *>(smem_raw);   // 3 planes of ROWS rows

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
    const int j0 = jt * TY + 1, k0 = zc * zchunk + 1;
    const int k1 = min(k0 + zchunk, n + 1);  // F on planes k0 .. k1-1
    const int i = (int)(threadIdx.x % RLN) + 1;
    const int rsub = (int)(threadIdx.x / RLN);
    const bool xin = i <= n;
    // element offsets inside one field fit in 32 bits (n <= 255)
    const int sy = (int)row_stride(n), sz = (int)plane_stride(n);
    const double *__restrict__ U = fp(u, qs);
    double *__restrict__ Fo = fp(F, qs);

    for (int r = threadIdx.x; r < 3 * ROWS; r += BLOCK) lp[r * RL] = 0.0;

    auto inside = [&](int j, int k) { return xin && j >= 1 && j <= n && k >= 1 && k <= n; };
    double pu[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = rsub + q * RPP, j = j0 - 1 + r;
        pu[q] = (r < ROWS && inside(j, k0 - 1)) ? U[i + j * sy + (k0 - 1) * sz] : 0.0;
    }
    double wm2[Q], wm1[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) wm2[q] = wm1[q] = 0.0;

    for (int k = k0 - 1; k <= k1; ++k) {
        double uk[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) uk[q] = pu[q];
        if (k < k1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int r = rsub + q * RPP, j = j0 - 1 + r;
                pu[q] = (r < ROWS && inside(j, k + 1)) ? U[i + j * sy + (k + 1) * sz] : 0.0;
            }
        }
        // ---- u plane k -> LDS
        double wn[Q];
        double *buf = lp + (k % 3 + 3) % 3 * ROWS * RL;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * RPP, j = j0 - 1 + r;
            const double v = (r < ROWS && inside(j, k)) ? uk[q] : 0.0;
            wn[q] = v;
            if (r < ROWS) buf[r * RL + i] = v;
        }
        __syncthreads();
        // ---- F on plane k-1 (three LDS buffers: plane k-1's buffer is not
        // rewritten before every thread has passed the next barrier)
        const int kb = k - 1;
        if (kb >= k0 && kb < k1) {
            const double *bb = lp + (kb % 3 + 3) % 3 * ROWS * RL;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int r = rsub + q * RPP, j = j0 - 1 + r;
                if (r >= 1 && r <= TY && j <= n && xin) {
                    const double *row = bb + r * RL;
                    double s = row[i - 1] + row[i + 1];
                    s += (bb[(r - 1) * RL + i] + bb[(r + 1) * RL + i]) + (wm2[q] + wn[q]);
                    s -= 6.0 * wm1[q];
                    Fo[i + j * sy + kb * sz] = cc * (ih2 * s);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            wm2[q] = wm1[q];
            wm1[q] = wn[q];
        }
    }
}

}  // namespace

namespace k {

// Small launches (a single 63^3 field of the coarse chain) take the
// column-blocked kernel: with few workgroups the z march is latency-bound.
bool apply_L_z_ok(const Tiling &t)
{
    if (t.dim != 3) return false;
    long points = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        if (t.seg_count(sg) > 0 && (t.seg_n(sg) < 31 || t.seg_n(sg) > 255)) return false;
        points += (long)t.seg_count(sg) * t.seg_n(sg) * t.seg_n(sg) * t.seg_n(sg);
    }
    return points >= (1L << 21);
}

hipError_t apply_L_z(const Tiling &t, double c, View<double> u, View<double> F, hipStream_t s)
{
    if (!apply_L_z_ok(t)) return hipErrorInvalidValue;
    int nmax = 0;
    long rows_total = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        nmax = std::max(nmax, t.seg_n(sg));
        rows_total += (long)t.seg_count(sg) * ((t.seg_n(sg) + TY - 1) / TY);
    }
    if (rows_total == 0) return hipSuccess;
    // z chunks: about 1024 workgroups in all, at least 4 planes each
    const long chunks = std::min<long>(std::max(1, nmax / 4), std::max<long>(1, (1024 + rows_total - 1) / rows_total));
    const int zchunk = (int)((nmax + chunks - 1) / chunks);
    long blocks = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        const int n = t.seg_n(sg);
        blocks += (long)t.seg_count(sg) * ((n + TY - 1) / TY) * ((n + zchunk - 1) / zchunk);
    }
    const int rln = nmax <= 64 ? 64 : nmax <= 128 ? 128 : 256;
    const size_t lds = (size_t)3 * (TY + 2) * (rln + 2) * sizeof(double);
    const dim3 g((unsigned)blocks), blk(BLOCK);
    if (rln == 64) return launch(apply_L_z_kernel<64, 2>, g, blk, lds, s, t, zchunk, c, u, F);
    if (rln == 128) return launch(apply_L_z_kernel<128, 3>, g, blk, lds, s, t, zchunk, c, u, F);
    return launch(apply_L_z_kernel<256, 6>, g, blk, lds, s, t, zchunk, c, u, F);
}

}  // namespace k
}  // namespace pfmg
