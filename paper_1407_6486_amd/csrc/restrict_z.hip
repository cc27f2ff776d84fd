// Residual plus full-weighting restriction in one pass over the fine grid
// (3D, fine n >= 63): bc = FW(b - (u - ah L u)), the coarse right-hand side
// of the V-cycle (Sec. 4.2.1; full weighting is the tensor product of the
// weights 1/4, 1/2, 1/4 around the fine point 2J of coarse point J).
//
// A workgroup owns TJ coarse rows of every coarse x and a chunk of coarse
// planes, and marches upwards through the fine planes 2K0-1 .. 2K1-1:
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

#include "kernels.h"

namespace pfmg {
namespace {

// RLN: x lanes per fine row (fine n rounded up to whole wavefronts).
// TJ coarse rows (at most 512 / RLN, so that the TJ x (RLN / 2) coarse
// points of a plane are at most one per thread); the 2 TJ + 1 fine residual
// rows are Q per thread.
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
    const int i = (int)(threadIdx.x % RLN) + 1;
    const int rsub = (int)(threadIdx.x / RLN);
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

    // x index 0 is the boundary: zero once in every LDS row
    for (int r = threadIdx.x; r < UR + FR; r += BLOCK) up[r * RL] = (T)0;

    auto inside = [&](int j, int k) { return xin && j >= 1 && j <= nf && k >= 1 && k <= nf; };
    auto ld = [&](const T *__restrict__ a, int j, int k) -> T {
        return inside(j, k) ? a[i + j * sy + k * sz] : (T)0;
    };
    // loads of step kf: u plane kf + 1 and b plane kf on the residual rows,
    // u plane kf on the two halo rows
    auto load_step = [&](int kf, T (&un)[Q], T (&bn)[Q], T (&ex)[2]) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * RPP;
            const bool own = r < FR;
            un[q] = own ? ld(U, fy0 + r, kf + 1) : (T)0;
            bn[q] = own ? ld(Bv, fy0 + r, kf) : (T)0;
        }
        ex[0] = ex[1] = (T)0;
        for (int e = rsub, q = 0; e < 2; e += RPP, ++q) ex[q] = ld(U, e == 0 ? fy0 - 1 : fy0 + FR, kf);
    };

    const int kf0 = 2 * K0 - 1, kf1 = 2 * K1 - 1;
    T um[Q], uc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = rsub + q * RPP;
        const bool own = r < FR;
        um[q] = own ? ld(U, fy0 + r, kf0 - 1) : (T)0;
        uc[q] = own ? ld(U, fy0 + r, kf0) : (T)0;
    }
    T pun[Q], pbn[Q], pex[2];
    load_step(kf0, pun, pbn, pex);
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    T acc = (T)0;

    for (int kf = kf0; kf <= kf1; ++kf) {
        T un[Q], bn[Q], ex[2];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            un[q] = pun[q];
            bn[q] = pbn[q];
        }
        ex[0] = pex[0];
        ex[1] = pex[1];
        if (kf < kf1) load_step(kf + 1, pun, pbn, pex);
        // ---- u plane kf -> LDS
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * RPP;
            if (r < FR) up[(r + 1) * RL + i] = uc[q];
        }
        for (int e = rsub, q = 0; e < 2; e += RPP, ++q) up[(e == 0 ? 0 : UR - 1) * RL + i] = ex[q];
        __syncthreads();
        // ---- residual of the tile's fine rows -> LDS
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = rsub + q * RPP;
            if (r < FR) {
                T res = (T)0;
                if (inside(fy0 + r, kf)) {
                    const T *row = up + (r + 1) * RL;
                    T s = row[i - 1] + row[i + 1];
                    s += (up[r * RL + i] + up[(r + 2) * RL + i]) + (um[q] + un[q]);
                    s -= (T)6 * uc[q];
                    res = bn[q] - (uc[q] - ah * s);
                }
                rp[r * RL + i] = res;
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
            if (kf & 1) {
                // fine plane 2K + 1 closes coarse plane K = (kf - 1) / 2 and
                // opens K + 1
                if (kf > kf0) C[(long)I + (long)J * syc + (long)((kf - 1) / 2) * szc] = acc + w[2] * s;
                acc = w[0] * s;
            } else {
                acc += w[1] * s;
            }
        }
        // ---- rotate the register windows
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            um[q] = uc[q];
            uc[q] = un[q];
        }
    }
}

}  // namespace

namespace k {

bool resid_restrict_z_ok(const Tiling &t)
{
    if (t.dim != 3) return false;
    for (int sg = 0; sg < t.nseg; ++sg)
        if (t.seg_count(sg) > 0 && (t.seg_n(sg) < 63 || t.seg_n(sg) > 255 || (t.seg_n(sg) & 1) == 0)) return false;
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
