// d-linear prolongation and correction in one z-marching pass (3D, odd fine
// n = 2 nc + 1 in [31, 255]): u += P ec, the coarse-grid correction of the
// V-cycle and the spatial interpolation of PFASST's coarse changes (Sec.
// 4.1.1, Sec. 2.4).  The fine value at 1-based (i, j, k) is the z-average of
// the bilinear in-plane values of coarse planes k >> 1 and (k + 1) >> 1 (one
// plane when k is even), each bilinear value the y-average of two x-averages
// (one point on an even axis); coarse index 0 and nc + 1 are the zero halo.
//
// A workgroup owns TYP fine rows of full x-rows and a chunk of coarse planes
// K = Ka .. Kb-1, and marches through them: at step K the coarse tile of
// plane K + 1 (the coarse rows under the workgroup's fine rows, every coarse
// x) goes to LDS, each thread forms the bilinear values of its fine points
// on that plane, and the fine planes 2K and 2K + 1 are corrected from the
// values of planes K and K + 1 held in registers.  Fine u is read and
// written once, each coarse value read once per workgroup: 16 + 1/8 x 8
// bytes per fine point in FP64.  The column kernel it replaces for large
// launches issued 16 coarse loads per 4 fine points; the arithmetic per
// point is the same, term for term.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace pfmg {
namespace {

constexpr int TYP = 8;   // fine rows per workgroup

// RLN: x lanes per fine row (fine n rounded up to whole wavefronts).
template <typename T, int RLN>
__global__ __launch_bounds__(BLOCK) void prolong_z_kernel(Tiling t, int kch, View<T> ec, View<T> u)
{
    constexpr int RPP = BLOCK / RLN;                 // fine rows per pass
    constexpr int Q = TYP / RPP;                     // fine rows per thread
    constexpr int CS = RLN / 2 + 2;                  // LDS row: coarse x = 0 .. RLN / 2 + 1
    constexpr int CR = TYP / 2 + 2;                  // coarse rows under TYP fine rows
    constexpr int NL = (CR * CS + BLOCK - 1) / BLOCK;  // tile loads per thread
    static_assert(Q * RPP == TYP, "rows per thread");
    extern __shared__ unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);       // two buffers of CR x CS

    unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [kch](int n) {
            return (long)((n + TYP - 1) / TYP) * ((coarser(n) + 1 + kch - 1) / kch);
        }))
        return;
    const int n = qs.n, nc = coarser(n);
    const int ytiles = (n + TYP - 1) / TYP, zch = (nc + 1 + kch - 1) / kch;
    const int item = (int)(bid / (unsigned)(ytiles * zch));
    const int rem = (int)(bid - (unsigned)item * (unsigned)(ytiles * zch));
    const int jt = rem / zch, zc = rem - jt * zch;
    if (mask && !mask[item]) return;
    qs.item = item;
    const int jf0 = jt * TYP + 1, cj0 = jf0 >> 1;
    const int Ka = zc * kch, Kb = min(Ka + kch, nc + 1);
    const int i = (int)(threadIdx.x % RLN) + 1;
    const int rsub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / RLN));
    const bool xin = i <= n;
    // element offsets inside one field fit in 32 bits (n <= 255)
    const int sy = (int)row_stride(n), sz = (int)plane_stride(n);
    const int csy = (int)row_stride(nc), csz = (int)plane_stride(nc);
    const T *__restrict__ E = fp(ec, qs);
    T *__restrict__ U = fp(u, qs);

    // coarse tile slots of this thread: LDS offset and clamped coarse offset
    int loff[NL], goff[NL];
    bool lok[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int idx = (int)threadIdx.x + l * BLOCK;
        lok[l] = idx < CR * CS;
        const int r = idx / CS, c = idx - r * CS;
        loff[l] = lok[l] ? idx : 0;
        goff[l] = min(cj0 + r, nc + 1) * csy + min(c, nc + 1);
    }
    auto load_tile = [&](int K, T (&v)[NL]) {
        const int pb = min(max(K, 0), nc + 1) * csz;
#pragma unroll
        for (int l = 0; l < NL; ++l) v[l] = E[pb + goff[l]];
    };
    auto store_tile = [&](T *buf, const T (&v)[NL]) {
#pragma unroll
        for (int l = 0; l < NL; ++l)
            if (lok[l]) buf[loff[l]] = v[l];
    };
    // per fine row (uniform): store flag, clamped row offset
    bool st[Q];
    int roff[Q], jr0[Q], jr1[Q];
    bool oy[Q];
    const int ii = min(i, n + 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = jf0 + rsub + q * RPP;
        st[q] = xin && j <= n;
        roff[q] = min(j, n + 1) * sy + ii;
        jr0[q] = (min(j, n) >> 1) - cj0;
        jr1[q] = ((min(j, n) + 1) >> 1) - cj0;
        oy[q] = (j & 1) != 0;
    }
    const int i0 = ii >> 1, i1 = min((ii + 1) >> 1, CS - 1);
    const bool ox = (i & 1) != 0;
    // bilinear value of this thread's fine point of row q on the tile
    auto bilin = [&](const T *buf, int q) -> T {
        const T *r0p = buf + jr0[q] * CS, *r1p = buf + jr1[q] * CS;
        const T c00 = r0p[i0], c01 = r0p[i1], c10 = r1p[i0], c11 = r1p[i1];
        const T r0 = ox ? (T)0.5 * (c00 + c01) : c00;
        const T r1 = ox ? (T)0.5 * (c10 + c11) : c10;
        return oy[q] ? (T)0.5 * (r0 + r1) : r0;
    };
    auto load_u = [&](int kf, T (&v)[Q]) {
        const int pb = min(max(kf, 0), n + 1) * sz;
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = U[pb + roff[q]];
    };

    // prologue: the bilinear values of plane Ka, the loads of step Ka
    T tn[NL], pa[Q], ue[Q], uo[Q];
    load_tile(Ka, tn);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __builtin_amdgcn_sched_barrier(0);
    store_tile(tile, tn);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) pa[q] = bilin(tile, q);
    load_tile(Ka + 1, tn);
    load_u(2 * Ka, ue);
    load_u(2 * Ka + 1, uo);

    for (int K = Ka; K < Kb; ++K) {
        // this step's loads were issued during the previous one
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __builtin_amdgcn_sched_barrier(0);
        T tc[NL], uec[Q], uoc[Q];
#pragma unroll
        for (int l = 0; l < NL; ++l) tc[l] = tn[l];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uec[q] = ue[q];
            uoc[q] = uo[q];
        }
        if (K + 1 < Kb) {
            load_tile(K + 2, tn);
            load_u(2 * K + 2, ue);
            load_u(2 * K + 3, uo);
        }
        // coarse plane K + 1 into the buffer the previous step did not read
        T *buf = tile + ((K - Ka + 1) & 1) * (CR * CS);
        store_tile(buf, tc);
        __syncthreads();
        const int ke = (2 * K) * sz, ko = (2 * K + 1) * sz;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const T pb = bilin(buf, q);
            if (st[q]) {
                // fine plane 2K (even: plane K alone; 2K = 0 is the halo)
                if (K >= 1) U[ke + roff[q]] = uec[q] + pa[q];
                // fine plane 2K + 1 (odd: planes K and K + 1)
                U[ko + roff[q]] = uoc[q] + (T)0.5 * (pa[q] + pb);
            }
            pa[q] = pb;
        }
    }
}

}  // namespace

namespace k {

bool prolong_z_ok(const Tiling &t)
{
    if (t.dim != 3) return false;
    long points = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        if (t.seg_count(sg) == 0) continue;
        const int n = t.seg_n(sg);
        if (n < 31 || n > 255 || (n & 1) == 0) return false;
        points += (long)t.seg_count(sg) * n * n * n;
    }
    // small launches (the coarse chain's single fields, four 31^3 fields)
    // stay on the column kernel: with few workgroups a z-march is
    // latency-bound
    return points >= (1L << 19);
}

template <typename T>
hipError_t prolong_z(const Tiling &t, View<T> ec, View<T> u, hipStream_t s, int kch_force)
{
    if (!prolong_z_ok(t)) return hipErrorInvalidValue;
    int nmax = 0;
    long rows_total = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        nmax = std::max(nmax, t.seg_n(sg));
        rows_total += (long)t.seg_count(sg) * ((t.seg_n(sg) + TYP - 1) / TYP);
    }
    if (rows_total == 0) return hipSuccess;
    const int ncmax = coarser(nmax);
    // coarse planes per chunk: about 2048 workgroups in all, at least two
    // chunks per field, at most 8 planes (measured at 127^3: 4 fields 24.2 us
    // with 2 planes, 20 fields 138 us with 8, 60 fields 432 us with 8 and
    // 445 us with 22)
    const long chunks = std::min<long>(ncmax + 1, std::max<long>(2, (2048 + rows_total - 1) / rows_total));
    const int kch =
        kch_force > 0 ? kch_force : std::min(8, (int)((ncmax + 1 + chunks - 1) / chunks));
    long blocks = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        const int n = t.seg_n(sg);
        blocks += (long)t.seg_count(sg) * ((n + TYP - 1) / TYP) * ((coarser(n) + 1 + kch - 1) / kch);
    }
    const int rln = nmax <= 64 ? 64 : nmax <= 128 ? 128 : 256;
    const size_t lds = (size_t)2 * (TYP / 2 + 2) * (rln / 2 + 2) * sizeof(T);
    const dim3 g((unsigned)blocks), blk(BLOCK);
    if (rln == 64) return launch(prolong_z_kernel<T, 64>, g, blk, lds, s, t, kch, ec, u);
    if (rln == 128) return launch(prolong_z_kernel<T, 128>, g, blk, lds, s, t, kch, ec, u);
    return launch(prolong_z_kernel<T, 256>, g, blk, lds, s, t, kch, ec, u);
}

template hipError_t prolong_z<double>(const Tiling &, View<double>, View<double>, hipStream_t, int);
template hipError_t prolong_z<float>(const Tiling &, View<float>, View<float>, hipStream_t, int);

}  // namespace k
}  // namespace pfmg
