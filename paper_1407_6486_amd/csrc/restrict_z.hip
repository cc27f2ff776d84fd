// Residual plus full-weighting restriction in one pass over the fine grid
// (3D, odd fine n >= 31): bc = FW(b - (u - ah L u)), the coarse right-hand side
// of the V-cycle (Sec. 4.2.1; full weighting is the tensor product of the
// weights 1/4, 1/2, 1/4 around the fine point 2J of coarse point J).
//
// A workgroup owns TJ coarse rows of every coarse x and a chunk of coarse
// planes, and marches through the fine planes 2K0-1 .. 2K1-1 (upwards in
// even chunks, downwards in odd ones, so that two neighbouring chunks read
// the planes they share at about the same time and the second read hits
// the XCD's L2):
//   1. the current fine plane of u goes to LDS (x and y neighbours; the z
//      neighbours stay in registers);
//   2. the residual of the 2 TJ + 1 fine rows of the tile goes to LDS,
//      every fine point once;
//   3. each thread folds its coarse point's 3 x 3 in-plane weights and adds
//      the plane, weighted by its z weight, to register accumulators: an
//      odd fine plane closes one coarse plane and opens the next.
// Fine u and b are read once (plus y-halo rows that neighbouring tiles also
// read), the coarse b written once: 16 + 1/8 x 8 bytes per fine point in
// FP64.  The loads of step kf + 1 are issued before step kf's arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace pfmg {
namespace {

// RLN: x lanes per fine row (fine n rounded up to whole wavefronts).
// TJ coarse rows (at most 512 / RLN, so that the TJ x (RLN / 2) coarse
// points of a plane are at most one per thread); the 2 TJ + 1 fine residual
// rows are Q per thread.
//
// As in the one-pass sweep, the march has no divergent branches around its
// loads: a thread's fine rows are wave-uniform, loads read clamped indices
// (zero halo words outside the interior), the interior test is a select,
// the register windows sit in slots indexed by the fine plane modulo 4 and
// the loop is unrolled four times; every step first waits for the loads of
// the previous step, then issues its own.
template <typename T, int RLN, int TJ>
__global__ __launch_bounds__(BLOCK) void resid_restrict_z_kernel(Tiling t, int kch, double alpha, View<T> b,
                                                                 View<T> u, View<T> bc)
{
    static_assert(TJ * RLN <= 512, "one coarse point per thread");
    constexpr int FR = 2 * TJ + 1;           // fine residual rows
    constexpr int UR = FR + 2;               // fine u rows in LDS (one halo row each side)
    constexpr int RPP = BLOCK / RLN;         // fine rows per pass of the workgroup
    constexpr int Q = (FR + RPP - 1) / RPP;  // fine rows per thread
    constexpr int RL = RLN + 2;              // LDS row: x = 0 .. RLN + 1
    constexpr int CX = RLN / 2;              // coarse x lanes
    extern __shared__ unsigned char smem_raw[];
    T *up = reinterpret_cast<T *>(smem_raw);  // LDS row e <-> fine row fy0 - 1 + e
    T *rp = up + UR * RL;             // LDS row r <-> fine row fy0 + r

    unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [kch](int nf) {
            const int nc = coarser(nf);
            return (long)((nc + TJ - 1) / TJ) * ((nc + kch - 1) / kch);
        }))
        return;
    const int nf = qs.n, nc = coarser(nf);
    const int ytiles = (nc + TJ - 1) / TJ, zch = (nc + kch - 1) / kch;
    const int item = (int)(bid / (unsigned)(ytiles * zch));
    const int rem = (int)(bid - (unsigned)item * (unsigned)(ytiles * zch));
    const int jt = rem / zch, zc = rem - jt * zch;
    if (mask && !mask[item]) return;
    qs.item = item;
    const T ah = (T)(qs.par(alpha) * (double)(nf + 1) * (double)(nf + 1));
    const int J0 = jt * TJ + 1, K0 = zc * kch + 1, K1 = min(K0 + kch, nc + 1);
    const int fy0 = 2 * J0 - 1;
    const int dk = (zc & 1) ? -1 : 1;   // march direction
    const int i = (int)(threadIdx.x % RLN) + 1;
    const int rsub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / RLN));
    const bool xin = i <= nf;
    // element offsets inside one field fit in 32 bits (n <= 255)
    const int sy = (int)row_stride(nf), sz = (int)plane_stride(nf);
    const T *__restrict__ U = fp(u, qs);
    const T *__restrict__ Bv = fp(b, qs);
    T *__restrict__ C = fp(bc, qs);
    const long syc = row_stride(nc), szc = plane_stride(nc);
    // this thread's coarse point
    const int I = (int)(threadIdx.x % CX) + 1, Jl = (int)(threadIdx.x / CX), J = J0 + Jl;
    const bool cin = I <= nc && Jl < TJ && J <= nc;
    // lanes past the row read its right halo word (zero)
    const unsigned ib = (unsigned)min(i, nf + 1) * (unsigned)sizeof(T);

    // x index 0 is the boundary: zero once in every LDS row
    for (int r = threadIdx.x; r < UR + FR; r += BLOCK) up[r * RL] = (T)0;

    // per fine row (uniform): ownership, clamped byte offset, interior lanes
    bool own[Q], rin[Q], eown[2];
    unsigned roff[Q], eoff[2];
    auto rowb = [&](int j) { return (unsigned)(min(max(j, 0), nf + 1) * sy) * (unsigned)sizeof(T); };
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = rsub + q * RPP, j = fy0 + r;
        own[q] = r < FR;
        roff[q] = rowb(j);
        rin[q] = xin && j >= 1 && j <= nf;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = rsub + q * RPP;
        eown[q] = e < 2;
        eoff[q] = rowb(e == 0 ? fy0 - 1 : fy0 + FR);
    }
    auto planeb = [&](int k) { return (unsigned)(min(max(k, 0), nf + 1) * sz) * (unsigned)sizeof(T); };
    auto ld = [&](const T *__restrict__ a, unsigned rb, unsigned pb) -> T {
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(a) + (rb + pb) + ib);
    };
    // loads of the step on plane kf: u plane kf + dk and b plane kf on the
    // residual rows, u plane kf on the two halo rows
    auto load_step = [&](int kf, T (&un)[Q], T (&bn)[Q], T (&ex)[2]) {
        const unsigned pu = planeb(kf + dk), pb = planeb(kf);
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (own[q]) {
                un[q] = ld(U, roff[q], pu);
                bn[q] = ld(Bv, roff[q], pb);
            }
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (eown[q]) ex[q] = ld(U, eoff[q], pb);
    };

    const int kf0 = 2 * K0 - 1, kf1 = 2 * K1 - 1;
    // step v = 0 .. L of the march works on fine plane kv(v); kf0 and kf1
    // are odd, so plane kv(v) is odd exactly when v is even in both
    // directions
    const int L = kf1 - kf0;
    auto kv = [&](int v) { return dk > 0 ? kf0 + v : kf1 - v; };
    // the plane of step v lives in slot (v + 1) & 3 (u), v & 1 (b, outer
    // halo rows)
    T us[4][Q], bs[2][Q], es[2][2];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
#pragma unroll
        for (int q = 0; q < Q; ++q) us[sl][q] = (T)0;
#pragma unroll
    for (int q = 0; q < Q; ++q) bs[0][q] = bs[1][q] = (T)0;
    es[0][0] = es[0][1] = es[1][0] = es[1][1] = (T)0;
    {
        const unsigned pm = planeb(kv(-1)), pc = planeb(kv(0));
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (own[q]) {
                us[0][q] = ld(U, roff[q], pm);
                us[1][q] = ld(U, roff[q], pc);
            }
    }
    load_step(kv(0), us[2], bs[0], es[0]);
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    // upwards: the running sum of the open coarse plane; downwards: the
    // weighted sums of its upper and middle fine planes, so that both
    // directions add the three planes in the same order
    T acc = (T)0, hi = (T)0, mid = (T)0;

    // step v = 4 m + S of the march, on fine plane kf = kv(v) (odd for
    // even S)
    auto step = [&](auto sc, int v) {
        constexpr int S = decltype(sc)::value;
        const int kf = kv(v);
        constexpr int SU = (S + 1) & 3;              // slot of u plane kf
        constexpr int SM = S & 3, SP = (S + 2) & 3, SN = (S + 3) & 3;
        // everything this step reads from memory was loaded during the
        // previous step: wait for it before issuing the next step's loads
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __builtin_amdgcn_sched_barrier(0);
        if (v < L) load_step(kf + dk, us[SN], bs[(S + 1) & 1], es[(S + 1) & 1]);
        // ---- u plane kf -> LDS
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * RPP;
            if (own[q]) up[(r + 1) * RL + i] = us[SU][q];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = rsub + q * RPP;
            if (eown[q]) up[(e == 0 ? 0 : UR - 1) * RL + i] = es[S & 1][q];
        }
        __syncthreads();
        // ---- residual of the tile's fine rows -> LDS
        const bool kin = kf >= 1 && kf <= nf;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * RPP;
            if (own[q]) {
                const T uc = us[SU][q];
                const T *row = up + (r + 1) * RL;
                T s = row[i - 1] + row[i + 1];
                s += (up[r * RL + i] + up[(r + 2) * RL + i]) + (us[SM][q] + us[SP][q]);
                s -= (T)6 * uc;
                const T res = bs[S & 1][q] - (uc - ah * s);
                rp[r * RL + i] = (kin && rin[q]) ? res : (T)0;
            }
        }
        __syncthreads();
        // ---- in-plane full weighting at this thread's coarse point
        if (cin) {
            T s = (T)0;
#pragma unroll
            for (int bq = -1; bq <= 1; ++bq) {
                const T *row = rp + (2 * Jl + 1 + bq) * RL + 2 * I;
                s += w[bq + 1] * ((w[0] * row[-1] + w[1] * row[0]) + w[2] * row[1]);
            }
            if (dk > 0) {
                if ((S & 1) == 0) {
                    // fine plane 2K + 1 closes coarse plane K = (kf - 1) / 2
                    // and opens K + 1
                    if (v > 0) C[(long)I + (long)J * syc + (long)((kf - 1) / 2) * szc] = acc + w[2] * s;
                    acc = w[0] * s;
                } else {
                    acc += w[1] * s;
                }
            } else {
                if ((S & 1) == 0) {
                    // fine plane 2K + 1 closes coarse plane K + 1 =
                    // (kf + 1) / 2 (its lower plane) and opens K
                    if (v > 0) {
                        T a = w[0] * s;
                        a += w[1] * mid;
                        C[(long)I + (long)J * syc + (long)((kf + 1) / 2) * szc] = a + w[2] * hi;
                    }
                    hi = s;
                } else {
                    mid = s;
                }
            }
        }
    };
    for (int vv = 0; vv <= L; vv += 4) {
        step(std::integral_constant<int, 0>{}, vv);
        if (vv + 1 > L) break;
        step(std::integral_constant<int, 1>{}, vv + 1);
        if (vv + 2 > L) break;
        step(std::integral_constant<int, 2>{}, vv + 2);
        if (vv + 3 > L) break;
        step(std::integral_constant<int, 3>{}, vv + 3);
    }
}

}  // namespace

namespace k {

bool resid_restrict_z_ok(const Tiling &t)
{
    if (t.dim != 3) return false;
    for (int sg = 0; sg < t.nseg; ++sg)
        if (t.seg_count(sg) > 0 && (t.seg_n(sg) < 31 || t.seg_n(sg) > 255 || (t.seg_n(sg) & 1) == 0)) return false;
    return true;
}

template <typename T>
hipError_t resid_restrict_z(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> bc, hipStream_t s)
{
    if (!resid_restrict_z_ok(t)) return hipErrorInvalidValue;
    int nmax = 0;
    for (int sg = 0; sg < t.nseg; ++sg) nmax = std::max(nmax, t.seg_n(sg));
    const int rln = nmax <= 64 ? 64 : nmax <= 128 ? 128 : 256;
    const int tj = 256 / rln;
    // coarse planes per chunk: about 2048 workgroups in all
    long rows_total = 0;
    for (int sg = 0; sg < t.nseg; ++sg) rows_total += (long)t.seg_count(sg) * ((coarser(t.seg_n(sg)) + tj - 1) / tj);
    if (rows_total == 0) return hipSuccess;
    const int ncmax = coarser(nmax);
    const long chunks = std::min<long>(ncmax, std::max<long>(1, (2048 + rows_total - 1) / rows_total));
    const int kch = (int)((ncmax + chunks - 1) / chunks);
    long blocks = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        const int nc = coarser(t.seg_n(sg));
        blocks += (long)t.seg_count(sg) * ((nc + tj - 1) / tj) * ((nc + kch - 1) / kch);
    }
    const int fr = 2 * tj + 1;
    const size_t lds = (size_t)(2 * fr + 2) * (rln + 2) * sizeof(T);
    const dim3 g((unsigned)blocks), blk(BLOCK);
    if (rln == 64) return launch(resid_restrict_z_kernel<T, 64, 4>, g, blk, lds, s, t, kch, alpha, b, u, bc);
    if (rln == 128) return launch(resid_restrict_z_kernel<T, 128, 2>, g, blk, lds, s, t, kch, alpha, b, u, bc);
    return launch(resid_restrict_z_kernel<T, 256, 1>, g, blk, lds, s, t, kch, alpha, b, u, bc);
}

template hipError_t resid_restrict_z<double>(const Tiling &, double, View<double>, View<double>, View<double>,
                                             hipStream_t);
template hipError_t resid_restrict_z<float>(const Tiling &, double, View<float>, View<float>, View<float>,
                                            hipStream_t);

}  // namespace k
}  // namespace pfmg
