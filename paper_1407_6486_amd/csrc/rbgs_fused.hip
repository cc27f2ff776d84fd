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
#include <type_traits>

#include "kernels.h"

namespace pfmg {
namespace {

constexpr int QMAX = 6;   // owned rows per thread

// One element at byte offset voff + soff of a buffer resource (soff uniform).
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, T v)
{
    if constexpr (sizeof(T) == 8) {
        using U2 = unsigned __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, (int)voff, (int)soff, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
    }
}

// RLN: x lanes per row (64, 128 or 256), the widest segment's n rounded up
// to whole wavefronts; narrower segments leave their extra lanes idle.
// NT: threads per workgroup (256 or 512: a larger workgroup owns more rows
// at the same register footprint, so fewer halo rows are re-read).
// Q: rows per thread, ceil((ty + 2) / (NT / RLN)) rounded up to an
// instantiated value; the register windows hold Q rows, so a small ty buys
// occupancy.  The loads of the next step are issued at the top of the
// current one (uin two planes ahead, b and the halo rows of uin one plane
// ahead) and
// wait behind the whole step's arithmetic and barriers.
//
// The z-march is written without divergent branches: a thread's rows are
// the same for the whole wavefront (RLN is a multiple of the wavefront
// width), so row and plane conditions are scalar; loads read clamped
// indices, whose values outside the interior are the zero halo words of
// the layout; the colour and the interior test pick results with selects.
// The register windows live in four slots indexed by the plane modulo 4
// and the loop is unrolled four times, so no values are moved between
// windows.
// TYC > 0 fixes the rows per workgroup at compile time (the shapes the
// shipped tuner table picks), which turns the row ownership tests into
// constants; TYC = 0 takes ty_rt.
template <typename T, int RLN, int Q, int NT, int TYC, int NB = 2>
__global__ __launch_bounds__(NT, (Q == 3 ? (NT == 256 ? 4 : 2) : 1)) void rbgs_fused_kernel(Tiling t, int ty_rt, int zchunk, int zero_in, double alpha,
                                                           double omega, View<T> b, View<T> uin, View<T> uout)
{
    extern __shared__ unsigned char smem_raw[];
    const int ty = TYC > 0 ? TYC : ty_rt;
    unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [&](int nn) {
            return (long)((nn + ty - 1) / ty) * ((nn + zchunk - 1) / zchunk);
        }))
        return;
    const int n = qs.n;
    constexpr int RL = RLN + 2;
    const int rows = ty + 2;                 // rows of the red update (owned rows)
    // uin plane k: rows j0-2 .. j0+ty+1 (NB = 1: two buffers, by the
    // plane's parity), then 2 planes of the red-updated field
    T *up0 = reinterpret_cast<T *>(smem_raw);
    T *wp = up0 + (NB == 1 ? 2 : 1) * (ty + 4) * RL;
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
    // odd z-chunks march downwards, so that two neighbouring chunks read
    // their shared border planes at the same time (both at their start or
    // both at their end) and the second read hits the XCD's L2.  Step v of
    // the march (v = -1 .. L) works on plane kv(v); the arithmetic is the
    // same in both directions (the z-neighbour sums commute).
    const int dk = (zc & 1) ? -1 : 1, L = k1 - k0;
    auto kv = [&](int v) { return dk > 0 ? k0 + v : k1 - 1 - v; };
    constexpr int rpp = NT / RLN;
    const int i = (int)(threadIdx.x % RLN) + 1;
    const int rsub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / RLN));
    __builtin_assume(rsub >= 0 && rsub < rpp);
    // element offsets inside one field fit in 32 bits (n <= 255)
    const int sy = (int)row_stride(n), sz = (int)plane_stride(n);
    const T *__restrict__ U = fp(uin, qs);
    const T *__restrict__ Bv = fp(b, qs);
    T *__restrict__ O = fp(uout, qs);
    const bool xin = i <= n;
    // lanes past the row read its right halo word (zero)
    const unsigned ib = (unsigned)min(i, n + 1) * (unsigned)sizeof(T);

    // x index 0 is the boundary: zero once in every LDS row
    for (int r = threadIdx.x; r < (NB == 1 ? 2 : 1) * (ty + 4) + 2 * rows; r += NT) up0[r * RL] = (T)0;

    // Per owned row (uniform): ownership, the byte offset of the row clamped
    // to the halo (every point outside the interior is zero), and the lanes
    // of the row that are red on even and on odd planes (interior only).
    bool own[Q], eown[2];
    unsigned roff[Q], eoff[2];
    // LEAN (rows of at most 128 lanes): the colours as wavefront lane masks
    // (scalar registers: picking one per plane is a scalar select), LDS
    // buffers picked by the step slot, buffer loads and stores; rows of 256
    // lanes keep per-lane booleans, buffers by plane parity and pointer
    // accesses, which measured faster there (193.6 against 203.6 us for an
    // FP32 sweep of 2 x 255^3, 387.8 against 396.9 us in FP64)
    constexpr bool LEAN = RLN <= 128;
    using Mask = std::conditional_t<LEAN, unsigned long long, bool>;
    Mask red_e[Q], red_o[Q];
    auto rowb = [&](int j) { return (unsigned)(min(max(j, 0), n + 1) * sy) * (unsigned)sizeof(T); };
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = rsub + q * rpp, j = j0 - 1 + r;
        own[q] = r < rows;
        roff[q] = rowb(j);
        const bool in = xin && j >= 1 && j <= n;
        const bool even = ((i + j) & 1) == 0;
        if constexpr (LEAN) {
            red_e[q] = __builtin_amdgcn_ballot_w64(in && even);
            red_o[q] = __builtin_amdgcn_ballot_w64(in && !even);
        } else {
            red_e[q] = in && even;
            red_o[q] = in && !even;
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = rsub + q * rpp;
        eown[q] = e < 2;
        eoff[q] = rowb(e == 0 ? j0 - 2 : j0 + ty + 1);
    }
    auto planeb = [&](int k) { return (unsigned)(min(max(k, 0), n + 1) * sz) * (unsigned)sizeof(T); };
    // loads and stores through buffer resources: the lane's byte offset is a
    // fixed vector register and the row and plane offset a scalar one, so
    // no address arithmetic runs on the vector unit
    const int fbytes = (int)(field_elems(n, 3) * (long)sizeof(T));
    const __amdgpu_buffer_rsrc_t rU = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(U), 0, fbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(Bv), 0, fbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rO = __builtin_amdgcn_make_buffer_rsrc(O, 0, fbytes, 0x00020000);
    auto ld = [&](__amdgpu_buffer_rsrc_t a, const T *__restrict__ ptr, unsigned rb, unsigned pb) -> T {
        if constexpr (LEAN)
            return buf_ld<T>(a, ib, rb + pb);
        else
            return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(ptr) + (rb + pb) + ib);
    };

    // The z-march; ZI: the input is zero (uin is not read).
    auto march = [&](auto zi) {
        constexpr bool ZI = decltype(zi)::value;
        // the global loads of the step on plane k: uin plane k + dk and b
        // plane k on the owned rows, uin plane k on the two outer halo rows
        auto load_step = [&](int k, T (&un)[Q], T (&bn)[Q], T (&ex)[2]) {
            const unsigned pu = planeb(k + dk), pb = planeb(k);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (own[q]) {
                    if (!ZI) un[q] = ld(rU, U, roff[q], pu);
                    bn[q] = ld(rB, Bv, roff[q], pb);
                }
            }
            if (!ZI) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    if (eown[q]) ex[q] = ld(rU, U, eoff[q], pb);
            }
        };

        T us[4][Q], bs[4][Q], ws[4][Q], es[2][2];
#pragma unroll
        for (int sl = 0; sl < 4; ++sl)
#pragma unroll
            for (int q = 0; q < Q; ++q) us[sl][q] = bs[sl][q] = ws[sl][q] = (T)0;
        es[0][0] = es[0][1] = es[1][0] = es[1][1] = (T)0;
        // the plane of step v lives in slot (v + 1) & 3 (uin, b, red field)
        // and (v + 1) & 1 (outer halo rows)
        if (!ZI) {
            const unsigned pm = planeb(kv(-2)), pc = planeb(kv(-1));
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (own[q]) {
                    us[3][q] = ld(rU, U, roff[q], pm);
                    us[0][q] = ld(rU, U, roff[q], pc);
                }
            }
        }
        load_step(kv(-1), us[1], bs[0], es[0]);

        // step v of the march, on plane k = kv(v), whose slot is S
        auto step = [&](auto sc, int v) {
            constexpr int S = decltype(sc)::value;
            const int k = kv(v);
            constexpr int S1 = (S + 1) & 3, S2 = (S + 2) & 3, S3 = (S + 3) & 3;
            // Everything this step reads from memory was loaded during the
            // previous step: wait for it here, before the next step's loads
            // are issued (a wait placed at the first use would also wait for
            // those, since how many are in flight depends on the row branches).
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            __builtin_amdgcn_sched_barrier(0);
            if (v < L) load_step(k + dk, us[S2], bs[S1], es[(S + 1) & 1]);
            // LDS buffers alternate with the step (slot parity), so their
            // offsets are compile-time constants
            T *up = up0 + (NB == 1 ? (LEAN ? (S & 1) : (k & 1)) * (ty + 4) * RL : 0);
            // ---- uin plane k -> LDS (rows e = 0 .. ty+3 <-> j = j0-2+e)
            if (!ZI) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int r = rsub + q * rpp;
                    if (own[q]) up[(r + 1) * RL + i] = us[S][q];
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int e = rsub + q * rpp;
                    if (eown[q]) up[(e == 0 ? 0 : ty + 3) * RL + i] = es[S & 1][q];
                }
            }
            // also orders phase B of the previous step (reading the red
            // plane buffer of k - 2 dk) before this step's red writes into it
            __syncthreads();
            // ---- phase A: red update of plane k on the owned rows
            T *wk = wp + (LEAN ? (S & 1) : (k & 1)) * rows * RL;
            const bool kin = k >= 1 && k <= n, kodd = (k & 1) != 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int r = rsub + q * rpp;
                if (own[q]) {
                    bool red;
                    if constexpr (LEAN)
                        red = __builtin_amdgcn_inverse_ballot_w64(kin ? (kodd ? red_o[q] : red_e[q]) : 0ull);
                    else
                        red = kin && (kodd ? red_o[q] : red_e[q]);
                    T val;
                    if (ZI) {
                        val = red ? winv * bs[S][q] : (T)0;
                    } else {
                        // outside the interior uc is a halo zero and stays
                        const T uc = us[S][q];
                        const T *row = up + (r + 1) * RL;
                        T s = row[i - 1] + row[i + 1];
                        s += (up[r * RL + i] + up[(r + 2) * RL + i]) + (us[S3][q] + us[S1][q]);
                        s -= (T)6 * uc;
                        const T upd = uc + winv * (bs[S][q] - (uc - ah * s));
                        val = red ? upd : uc;
                    }
                    ws[S][q] = val;
                    wk[r * RL + i] = val;
                }
            }
            // NB = 2: the uin plane buffer is rewritten by the next step, so
            // phase A must be done everywhere first.  NB = 1: the next step
            // writes the other uin buffer, and phase B below reads only the
            // red plane of the previous step (ordered by this step's first
            // barrier), so that barrier alone orders every LDS access.
            if constexpr (NB == 2) __syncthreads();
            // ---- phase B: black update of plane k - dk on rows 1..ty
            const int kb = k - dk;
            if (kb >= k0 && kb < k1) {
                const T *wb = wp + (LEAN ? ((S + 1) & 1) : (kb & 1)) * rows * RL;
                const bool kbodd = (kb & 1) != 0;
                T outv[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int r = rsub + q * rpp;
                    outv[q] = (T)0;
                    if (r >= 1 && r <= ty) {
                        bool black;
                        if constexpr (LEAN)
                            black = __builtin_amdgcn_inverse_ballot_w64(kbodd ? red_e[q] : red_o[q]);
                        else
                            black = kbodd ? red_e[q] : red_o[q];
                        const T wc = ws[S3][q];
                        const T *row = wb + r * RL;
                        T s = row[i - 1] + row[i + 1];
                        s += (wb[(r - 1) * RL + i] + wb[(r + 1) * RL + i]) + (ws[S2][q] + ws[S][q]);
                        s -= (T)6 * wc;
                        const T upd = wc + winv * (bs[S3][q] - (wc - ah * s));
                        outv[q] = black ? upd : wc;
                    }
                }
                if (xin) {
                    const unsigned pk = planeb(kb);
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int r = rsub + q * rpp;
                        const int j = j0 - 1 + r;
                        if (r >= 1 && r <= ty && j <= n) {
                            if constexpr (LEAN)
                                buf_st<T>(rO, ib, roff[q] + pk, outv[q]);
                            else
                                O[i + j * sy + kb * sz] = outv[q];
                        }
                    }
                }
            }
        };
        for (int vv = -1; vv <= L; vv += 4) {
            step(std::integral_constant<int, 0>{}, vv);
            if (vv + 1 > L) break;
            step(std::integral_constant<int, 1>{}, vv + 1);
            if (vv + 2 > L) break;
            step(std::integral_constant<int, 2>{}, vv + 2);
            if (vv + 3 > L) break;
            step(std::integral_constant<int, 3>{}, vv + 3);
        }
    };
    if (zero_in)
        march(std::true_type{});
    else
        march(std::false_type{});
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
#define PFMG_FUSED_TY(RL_, Q_, NT_, TY_)                                                                         \
    return launch(rbgs_fused_kernel<T, RL_, Q_, NT_, TY_>, g, blk, f.lds, s, t, f.ty, f.zchunk, zi, alpha, omega, b, \
                  uin, uout)
#define PFMG_FUSED(RL_, Q_, NT_) PFMG_FUSED_TY(RL_, Q_, NT_, 0)
    // compile-time rows for the shapes of the 127^3 / 63^3 / 31^3 V-cycle
    // levels in the shipped FP64 tuner table
    if constexpr (sizeof(T) == 8) {
        if (f.nt == 512 && rln == 128 && q == 3 && f.ty == 8) {
            // one barrier per z-step (the uin plane double-buffered in LDS):
            // 41.0 us against 41.4 us for 4 x 127^3 at 0.3 more KB per row
            // (read at every launch, so a caller can compare the two)
            const bool one_barrier = env_int("PFMG_SWEEP_1B", 1) != 0;
            if (one_barrier)
                return launch(rbgs_fused_kernel<T, 128, 3, 512, 8, 1>, g, blk,
                              f.lds + (size_t)(f.ty + 4) * (rln + 2) * sizeof(T), s, t, f.ty, f.zchunk, zi, alpha,
                              omega, b, uin, uout);
            PFMG_FUSED_TY(128, 3, 512, 8);
        }
        if (f.nt == 512 && rln == 64 && q == 2 && f.ty == 8) PFMG_FUSED_TY(64, 2, 512, 8);
        if (f.nt == 512 && rln == 64 && q == 3 && f.ty == 16) PFMG_FUSED_TY(64, 3, 512, 16);
        if (f.nt == 512 && rln == 64 && q == 1 && f.ty == 6) PFMG_FUSED_TY(64, 1, 512, 6);
        if (f.nt == 256 && rln == 64 && q == 1 && f.ty == 2) PFMG_FUSED_TY(64, 1, 256, 2);
    }
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
#undef PFMG_FUSED_TY
    return hipErrorInvalidValue;
}

template hipError_t rbgs_fused<double>(const Tiling &, double, double, bool, View<double>, View<double>,
                                       View<double>, hipStream_t, const FusedShape *);
template hipError_t rbgs_fused<float>(const Tiling &, double, double, bool, View<float>, View<float>, View<float>,
                                      hipStream_t, const FusedShape *);

}  // namespace k
}  // namespace pfmg
