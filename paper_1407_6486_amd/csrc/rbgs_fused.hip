// One whole red-black Gauss-Seidel sweep in one pass over HBM (3D).
//
// uout = RBGS(uin, b): red points (1-based i+j+k even) first, each from the
// old black neighbours, then black points from the new red ones (the
// smoother of Sec. 4.2.1; weight omega, omega = 1 is plain Gauss-Seidel).
// Out of place, so uin and b are read once and uout written once:
// 24 bytes per point in FP64 instead of 2 x 24 for two in-place colour
// passes whose interleaved colours waste half of every cache line.
//
// A workgroup owns full x-rows (the x boundary is the only x halo), `ty`
// output rows and a chunk of z planes, and marches upwards in z.  At step k
//   A: red update of plane k on rows j0-1 .. j0+ty (one halo row each side
//      is recomputed, so workgroups never exchange data);
//   B: black update of plane k-1 on rows j0 .. j0+ty-1, written out with the
//      red values of that plane.
// Each thread owns the same rows in both phases and keeps its column's
// values of the neighbouring planes in registers: uin at k-1, k, k+1, the
// red-updated field at k-2, k-1, k and b at k-1, k.  Only the current plane
// of uin and of the red-updated field pass through LDS, for the x and y
// neighbours.  Every global load of a step is issued before its barrier.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "kernels.h"

namespace pfmg {
namespace {

constexpr int QMAX = 6;   // owned rows per thread

// RLN: x lanes per row (64, 128 or 256), the widest segment's n rounded up
// to whole wavefronts; narrower segments leave their extra lanes idle.
// NT: threads per workgroup (256 or 512: a larger workgroup owns more rows
// at the same register footprint, so fewer halo rows are re-read).
// Q: rows per thread, ceil((ty + 2) / (NT / RLN)) rounded up to an
// instantiated value; the register windows hold Q rows, so a small ty buys
// occupancy.  The loads of step k + 1 are issued at the top of step k
// (uin plane k + 2, b plane k + 1, the halo rows of uin plane k + 1) and
// wait behind the whole step's arithmetic and barriers.
template <typename T, int RLN, int Q, int NT>
__global__ __launch_bounds__(NT, (Q == 3 ? (NT == 256 ? 5 : 2) : 1)) void rbgs_fused_kernel(Tiling t, int ty, int zchunk, int zero_in, double alpha,
                                                           double omega, View<T> b, View<T> uin, View<T> uout)
{
    extern __shared__ unsigned char smem_raw[];
    unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [ty, zchunk](int nn) {
            return (long)((nn + ty - 1) / ty) * ((nn + zchunk - 1) / zchunk);
        }))
        return;
    const int n = qs.n;
    constexpr int rowlanes = RLN;
    constexpr int RL = rowlanes + 2;
    const int rows = ty + 2;                 // rows of the red update (owned rows)
    T *up = reinterpret_cast<T *>(smem_raw);             // uin plane k: rows j0-2 .. j0+ty+1
    T *wp = up + (ty + 4) * RL;                  // 2 planes of the red-updated field
    const int ytiles = (n + ty - 1) / ty, zch = (n + zchunk - 1) / zchunk;
    const int item = (int)(bid / (unsigned)(ytiles * zch));
    const int rem = (int)(bid - (unsigned)item * (unsigned)(ytiles * zch));
    const int jt = rem / zch, zc = rem - jt * zch;
    if (mask && !mask[item]) return;
    qs.item = item;
    const double ahd = qs.par(alpha) * (double)(n + 1) * (double)(n + 1);
    const T ah = (T)ahd, winv = (T)(omega / (1.0 + 2.0 * 3 * ahd));
    const int j0 = jt * ty + 1, k0 = zc * zchunk + 1;
    const int k1 = min(k0 + zchunk, n + 1);
    constexpr int rpp = NT / rowlanes;
    const int i = (int)(threadIdx.x % rowlanes) + 1;
    const int rsub = (int)(threadIdx.x / rowlanes);
    // element offsets inside one field fit in 32 bits (n <= 255)
    const int sy = (int)row_stride(n), sz = (int)plane_stride(n);
    const T *__restrict__ U = fp(uin, qs);
    const T *__restrict__ Bv = fp(b, qs);
    T *__restrict__ O = fp(uout, qs);
    const bool xin = i <= n;

    // x index 0 is the boundary: zero once in every LDS row
    for (int r = threadIdx.x; r < (ty + 4) + 2 * rows; r += NT) up[r * RL] = (T)0;

    auto inside = [&](int j, int k) { return xin && j >= 1 && j <= n && k >= 1 && k <= n; };
    auto ld = [&](const T *__restrict__ a, int j, int k) -> T {
        return inside(j, k) ? a[i + j * sy + k * sz] : (T)0;
    };
    // the global loads of step k
    auto load_step = [&](int k, T (&un)[Q], T (&bn)[Q], T (&ex)[2]) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * rpp;
            const int j = j0 - 1 + r;
            const bool own = r < rows;
            un[q] = (own && !zero_in) ? ld(U, j, k + 1) : (T)0;
            bn[q] = own ? ld(Bv, j, k) : (T)0;
        }
        ex[0] = ex[1] = (T)0;
        if (!zero_in)
            for (int e = rsub, q = 0; e < 2; e += rpp, ++q) ex[q] = ld(U, e == 0 ? j0 - 2 : j0 + ty + 1, k);
    };

    T um[Q], uc[Q], wm2[Q], wm1[Q], bm1[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = rsub + q * rpp;
        const int j = j0 - 1 + r;
        const bool own = r < rows;
        um[q] = (own && !zero_in) ? ld(U, j, k0 - 2) : (T)0;
        uc[q] = (own && !zero_in) ? ld(U, j, k0 - 1) : (T)0;
        wm2[q] = wm1[q] = bm1[q] = (T)0;
    }
    T pun[Q], pbn[Q], pex[2];
    load_step(k0 - 1, pun, pbn, pex);

    for (int k = k0 - 1; k <= k1; ++k) {
        T un[Q], bn[Q], ex[2];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            un[q] = pun[q];
            bn[q] = pbn[q];
        }
        ex[0] = pex[0];
        ex[1] = pex[1];
        if (k < k1) load_step(k + 1, pun, pbn, pex);
        // ---- uin plane k -> LDS (rows e = 0 .. ty+3 <-> j = j0-2+e)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * rpp;
            if (r < rows) up[(r + 1) * RL + i] = uc[q];
        }
        for (int e = rsub, q = 0; e < 2; e += rpp, ++q) up[(e == 0 ? 0 : ty + 3) * RL + i] = ex[q];
        __syncthreads();
        // ---- phase A: red update of plane k on the owned rows
        T *wk = wp + (k & 1) * rows * RL;
        T wn[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * rpp;
            const int j = j0 - 1 + r;
            T val = (T)0;
            if (r < rows && inside(j, k)) {
                const bool red = ((i + j + k) & 1) == 0;
                if (zero_in) {
                    val = red ? winv * bn[q] : (T)0;
                } else if (red) {
                    const T *row = up + (r + 1) * RL;
                    T s = row[i - 1] + row[i + 1];
                    s += (up[r * RL + i] + up[(r + 2) * RL + i]) + (um[q] + un[q]);
                    s -= (T)6 * uc[q];
                    val = uc[q] + winv * (bn[q] - (uc[q] - ah * s));
                } else {
                    val = uc[q];
                }
            }
            wn[q] = val;
            if (r < rows) wk[r * RL + i] = val;
        }
        __syncthreads();
        // ---- phase B: black update of plane k-1 on rows 1..ty
        const int kb = k - 1;
        if (kb >= k0 && kb < k1) {
            const T *wb = wp + (kb & 1) * rows * RL;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int r = rsub + q * rpp;
                const int j = j0 - 1 + r;
                if (r >= 1 && r <= ty && j <= n && xin) {
                    const T wc = wm1[q];
                    T out = wc;
                    if (((i + j + kb) & 1) == 1) {
                        const T *row = wb + r * RL;
                        T s = row[i - 1] + row[i + 1];
                        s += (wb[(r - 1) * RL + i] + wb[(r + 1) * RL + i]) + (wm2[q] + wn[q]);
                        s -= (T)6 * wc;
                        out = wc + winv * (bm1[q] - (wc - ah * s));
                    }
                    O[i + j * sy + kb * sz] = out;
                }
            }
        }
        // ---- rotate the register windows
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            um[q] = uc[q];
            uc[q] = un[q];
            wm2[q] = wm1[q];
            wm1[q] = wn[q];
            bm1[q] = bn[q];
        }
    }
}

// Rows per thread for a launch of row width RLN and ty output rows.
constexpr int rows_per_thread(int rln, int ty, int nt) { return (ty + 2 + nt / rln - 1) / (nt / rln); }

int env_int(const char *name, int dflt)
{
    const char *e = getenv(name);
    return e ? atoi(e) : dflt;
}

}  // namespace

namespace k {

bool rbgs_fused_ty_ok(int nmax, int ty, int nt)
{
    if (nmax < 1 || nmax > 256 || ty < 1 || (nt != 256 && nt != 512)) return false;
    const int rln = (nmax + 63) & ~63;
    // 512-thread workgroups are instantiated for up to 3 rows per thread
    return rows_per_thread(rln, ty, nt) <= (nt == 512 ? 3 : QMAX);
}

// Rows per workgroup and planes per z-chunk for a launch over the grids of
// `t` (the same shape for every segment; LDS sized for the widest rows).
// ty / target_blocks = 0 take the defaults (8 rows, 4 for 256-lane rows;
// about 1024 workgroups); nt: 256 or 512 threads per workgroup; ty is
// halved until every thread owns at most the instantiated row count (QMAX,
// 3 for 512 threads).
FusedShape rbgs_fused_shape(const Tiling &t, size_t elem, int ty, int target_blocks, int nt)
{
    int nmax = 0;
    long rows_total = 0;
    for (int sg = 0; sg < t.nseg; ++sg) nmax = std::max(nmax, t.seg_n(sg));
    const int rowlanes = (nmax + 63) & ~63;
    FusedShape f;
    f.nt = nt == 512 ? 512 : 256;
    f.ty = ty > 0 ? ty : env_int("PFMG_RB_TY", rowlanes >= 256 ? 4 : 8);
    while (f.ty > 1 && !rbgs_fused_ty_ok(nmax, f.ty, f.nt)) f.ty /= 2;
    for (int sg = 0; sg < t.nseg; ++sg) rows_total += (long)t.seg_count(sg) * ((t.seg_n(sg) + f.ty - 1) / f.ty);
    const int target = target_blocks > 0 ? target_blocks : env_int("PFMG_RB_BLOCKS", 1024);
    int zch = (int)std::min<long>(std::max<long>(1, (target + rows_total - 1) / std::max(1L, rows_total)),
                                  std::max(1, nmax / 4));
    f.zchunk = target_blocks > 0 ? (nmax + zch - 1) / zch : env_int("PFMG_RB_ZCH", (nmax + zch - 1) / zch);
    f.blocks = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        const int n = t.seg_n(sg);
        f.blocks += (long)t.seg_count(sg) * ((n + f.ty - 1) / f.ty) * ((n + f.zchunk - 1) / f.zchunk);
    }
    f.lds = (size_t)((f.ty + 4) + 2 * (f.ty + 2)) * (rowlanes + 2) * elem;
    return f;
}

template <typename T>
hipError_t rbgs_fused(const Tiling &t, double alpha, double omega, bool zero_in, View<T> b, View<T> uin,
                      View<T> uout, hipStream_t s, const FusedShape *shape)
{
    if (t.dim != 3) return hipErrorInvalidValue;
    for (int sg = 0; sg < t.nseg; ++sg)
        if (t.seg_n(sg) < 31 || t.seg_n(sg) > 255) return hipErrorInvalidValue;
    const FusedShape f = shape ? *shape : rbgs_fused_shape(t, sizeof(T));
    // the kernel derives its tiles from ty and zchunk: reject shapes the
    // launch does not cover exactly
    const FusedShape chk = rbgs_fused_shape(t, sizeof(T), f.ty, 1, f.nt);
    long blocks = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        const int n = t.seg_n(sg);
        blocks += (long)t.seg_count(sg) * ((n + f.ty - 1) / f.ty) * ((n + f.zchunk - 1) / f.zchunk);
    }
    if (f.ty < 1 || f.ty != chk.ty || f.zchunk < 1 || blocks != f.blocks || f.lds != chk.lds || f.nt != chk.nt)
        return hipErrorInvalidValue;
    if (f.blocks == 0) return hipSuccess;
    int nmax = 0;
    for (int sg = 0; sg < t.nseg; ++sg) nmax = std::max(nmax, t.seg_n(sg));
    const int zi = zero_in ? 1 : 0;
    const int rln = nmax <= 64 ? 64 : nmax <= 128 ? 128 : 256;
    const int q = rows_per_thread(rln, f.ty, f.nt);
    const dim3 g((unsigned)f.blocks), blk(f.nt);
#define PFMG_FUSED(RL_, Q_, NT_)                                                                                \
    return launch(rbgs_fused_kernel<T, RL_, Q_, NT_>, g, blk, f.lds, s, t, f.ty, f.zchunk, zi, alpha, omega, b, uin, \
                  uout)
    // instantiated row counts: those of ty = 1, 2, 4, 8, 16 that fit QMAX,
    // and QMAX for any other ty; 512-thread workgroups for up to 3 rows
    if (f.nt == 512) {
        if (rln == 64) {
            if (q <= 1) PFMG_FUSED(64, 1, 512);
            if (q <= 2) PFMG_FUSED(64, 2, 512);
            if (q <= 3) PFMG_FUSED(64, 3, 512);
        } else if (rln == 128) {
            if (q <= 2) PFMG_FUSED(128, 2, 512);
            if (q <= 3) PFMG_FUSED(128, 3, 512);
        } else {
            if (q <= 3) PFMG_FUSED(256, 3, 512);
        }
        return hipErrorInvalidValue;
    }
    if (rln == 64) {
        if (q <= 1) PFMG_FUSED(64, 1, 256);
        if (q <= 2) PFMG_FUSED(64, 2, 256);
        if (q <= 3) PFMG_FUSED(64, 3, 256);
        if (q <= 5) PFMG_FUSED(64, 5, 256);
        if (q <= QMAX) PFMG_FUSED(64, 6, 256);
    } else if (rln == 128) {
        if (q <= 2) PFMG_FUSED(128, 2, 256);
        if (q <= 3) PFMG_FUSED(128, 3, 256);
        if (q <= 5) PFMG_FUSED(128, 5, 256);
        if (q <= QMAX) PFMG_FUSED(128, 6, 256);
    } else {
        if (q <= 3) PFMG_FUSED(256, 3, 256);
        if (q <= 4) PFMG_FUSED(256, 4, 256);
        if (q <= QMAX) PFMG_FUSED(256, 6, 256);
    }
#undef PFMG_FUSED
    return hipErrorInvalidValue;
}

template hipError_t rbgs_fused<double>(const Tiling &, double, double, bool, View<double>, View<double>,
                                       View<double>, hipStream_t, const FusedShape *);
template hipError_t rbgs_fused<float>(const Tiling &, double, double, bool, View<float>, View<float>, View<float>,
                                      hipStream_t, const FusedShape *);

}  // namespace k
}  // namespace pfmg
