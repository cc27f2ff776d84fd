// SDC, FAS and collocation-residual kernels on gfx950 (FP64).
//
//  apply_L       F = nu L_h u, the right-hand side of the semi-discrete
//                heat equation at one node (Sec. 4.1 / 4.2).
//  sdc_integrals I_m = dt sum_i (q_{m+1,i} - q_{m,i}) F_i (eq. sdc-be),
//                all M node-to-node integrals of one slice in one pass.
//  sdc_rhs       right-hand side of the node solve of eq. SDCcompactLIII in
//                node-to-node form, plus the FAS difference on level 1.
//  sdc_start     the start of a sweep in one pass: node 0 taken from a
//                source (the previous slice's last node) when given, all
//                integrals, and the first node solve's right-hand side.
//  apply_L_rhs   F at one node and the next node solve's right-hand side
//                from the same loads (column-blocked small launches).
//  solve_F_rhs   F at one node from its solve, (u - b) / delta, and the
//                next node solve's right-hand side in the same pass.
//  fas_inject /  FAS coarsening (Sec. 2.3): point-wise injection of U and
//  fas_tau       of the fine node integrals dt Q_f F_f, minus the coarse
//                integrals dt Q_c F_c of the injected state.
//  interp_coarse coarse corrections combined by Lagrange interpolation in
//                time; the spatial part is the prolongation kernel.
//  colloc_resid  eq. resid, max-norm per slice.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "kernels.h"

namespace pfmg {
namespace {

constexpr int MAXN = 16;   // nodes per slice upper bound


template <int DIM>
__global__ __launch_bounds__(BLOCK) void apply_L_kernel(Tiling t, double c, View<double> u, View<double> F)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const double *uu = fp(u, q);
    const double ih2 = (double)(q.n + 1) * (double)(q.n + 1);
    fp(F, q)[o] = q.par(c) * (ih2 * d2sum<DIM>(uu, o, row_stride(q.n), plane_stride(q.n)));
}

// Column-blocked 3D variant (KZ planes per thread, loads before stores).
constexpr int KZ = 4;
__global__ __launch_bounds__(BLOCK) void apply_L_kz_kernel(Tiling t, double c, View<double> u, View<double> F)
{
    Pt q; int i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, q, i, j, k0, nk, o)) return;
    const long sy = row_stride(q.n), sz = plane_stride(q.n);
    const double *__restrict__ uu = fp(u, q);
    double *__restrict__ ff = fp(F, q);
    const double ih2 = (double)(q.n + 1) * (double)(q.n + 1);
    const double cc = q.par(c);
    // every load unguarded (a short column repeats its last plane)
    double col[KZ + 2], xs[KZ], ys[KZ];
#pragma unroll
    for (int w = 0; w < KZ + 2; ++w) col[w] = uu[o + (long)(min(w, nk + 1) - 1) * sz];
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        const long ow = o + (long)min(w, nk - 1) * sz;
        xs[w] = uu[ow - 1] + uu[ow + 1];
        ys[w] = uu[ow - sy] + uu[ow + sy];
    }
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        if (w < nk) {
            double s = xs[w];
            s += ys[w] + (col[w] + col[w + 2]);
            s -= 6.0 * col[w + 1];
            ff[o + (long)w * sz] = cc * (ih2 * s);
        }
    }
}

// NN > 0 fixes the node count at compile time (node values stay in
// registers); NN == 0 is the generic path for any count up to MAXN.
// Per-field scalars (dt, delta) come from the segment when it has them.
template <int DIM, int NN>
__global__ __launch_bounds__(BLOCK) void sdc_integrals_kernel(Tiling t, int nn_rt, double dt, const double *__restrict__ S,
                                                              View<double> F, View<double> I)
{
    const int nn = NN > 0 ? NN : nn_rt;
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const long f_node = node_stride(q.n, DIM), i_node = f_node;
    const double h = q.par(dt);
    const double *f = fp(F, q) + o;
    double fv[MAXN];
    for (int w = 0; w < nn; ++w) fv[w] = f[w * f_node];
    double *out = fp(I, q) + o;
    for (int m = 0; m + 1 < nn; ++m) {
        double acc = 0.0;
        for (int w = 0; w < nn; ++w) acc += S[m * nn + w] * fv[w];
        out[m * i_node] = h * acc;
    }
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void sdc_rhs_kernel(Tiling t, double delta, View<double> Um, View<double> Fm1,
                                                        View<double> Im, View<double> t1, View<double> t0, View<double> b)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    // every load first (without t1 the difference reads Um twice, unused)
    const bool ht = t1.p != nullptr;
    const double *um = fp(Um, q);
    const double um_v = um[o], fm = fp(Fm1, q)[o], im = fp(Im, q)[o];
    const double x1 = (ht ? fp(t1, q) : um)[o], x0 = (ht ? fp(t0, q) : um)[o];
    double v = um_v - q.par(delta) * fm + im;
    if (ht) v = v + (x1 - x0);
    fp(b, q)[o] = v;
}

// F = (u - b) / delta at the node just solved (b still holds its
// right-hand side), then, with Fn1 set, b = u - delta_next Fn1 + In
// (+ t1 - t0): the next node's right-hand side, as in sdc_rhs.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void solve_F_rhs_kernel(Tiling t, double delta, View<double> U, View<double> B,
                                                            View<double> F, double delta_next, View<double> Fn1,
                                                            View<double> In, View<double> t1, View<double> t0)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    // every load before the first store (absent arrays read U, unused)
    const double *uu = fp(U, q);
    double *bb = fp(B, q);
    const bool hn = Fn1.p != nullptr, ht = t1.p != nullptr;
    const double u = uu[o], bo = bb[o];
    const double fn = (hn ? fp(Fn1, q) : uu)[o], in = (hn ? fp(In, q) : uu)[o];
    const double x1 = (hn && ht ? fp(t1, q) : uu)[o], x0 = (hn && ht ? fp(t0, q) : uu)[o];
    fp(F, q)[o] = (u - bo) / q.par(delta);
    if (!hn) return;
    double v = u - q.par(delta_next) * fn + in;
    if (ht) v = v + (x1 - x0);
    bb[o] = v;
}

// sdc_integrals followed by sdc_rhs for the first node, with the same
// arithmetic; with Usrc / Fsrc set, node 0 of U and F is first copied from
// them (the send-forward of the coarse chain and of the predictor rounds).
template <int DIM, int NN>
__global__ __launch_bounds__(BLOCK) void sdc_start_kernel(Tiling t, int nn_rt, double dt, const double *__restrict__ S,
                                                          double delta1, View<double> U, View<double> F,
                                                          View<double> Usrc, View<double> Fsrc, View<double> I,
                                                          View<double> tau, View<double> b, double nu0)
{
    const int nn = NN > 0 ? NN : nn_rt;
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const long f_node = node_stride(q.n, DIM);
    const double h = q.par(dt);
    double *u = fp(U, q) + o;
    double *f = fp(F, q) + o;
    // every load before the first store: the other nodes' F and tau (read
    // from F when absent, unused) first, then node 0
    const bool ht = tau.p != nullptr;
    const double *tb = ht ? fp(tau, q) + o : f;
    double fv[MAXN];
    for (int w = 1; w < nn; ++w) fv[w] = f[w * f_node];
    const double t_hi = tb[f_node], t_lo = tb[0];
    double u0;
    if (Usrc.p) {
        const double *us = fp(Usrc, q);
        u0 = us[o];
        if (nu0 > 0.0) {
            // F of the new node 0 evaluated from its value (apply_L's arithmetic)
            const double ih2 = (double)(q.n + 1) * (double)(q.n + 1);
            fv[0] = q.par(nu0) * (ih2 * d2sum<DIM>(us, o, row_stride(q.n), plane_stride(q.n)));
        } else {
            fv[0] = fp(Fsrc, q)[o];
        }
    } else {
        u0 = u[0];
        fv[0] = f[0];
    }
    if (Usrc.p) {
        u[0] = u0;
        f[0] = fv[0];
    }
    double *out = fp(I, q) + o;
    double i0 = 0.0;
    for (int m = 0; m + 1 < nn; ++m) {
        double acc = 0.0;
        for (int w = 0; w < nn; ++w) acc += S[m * nn + w] * fv[w];
        const double v = h * acc;
        out[m * f_node] = v;
        if (m == 0) i0 = v;
    }
    double v = u0 - q.par(delta1) * fv[1] + i0;
    if (ht) v = v + (t_hi - t_lo);
    fp(b, q)[o] = v;
}

// apply_L_kz plus, from the same column loads, the next node solve's
// right-hand side b = u - delta Fn1 + In (+ t1 - t0), the sdc_rhs
// arithmetic (Fn1: the old F of the next node, In its integral).
__global__ __launch_bounds__(BLOCK) void apply_L_rhs_kz_kernel(Tiling t, double c, View<double> u, View<double> F,
                                                               double delta, View<double> Fn1, View<double> In,
                                                               View<double> t1, View<double> t0, View<double> b)
{
    Pt q; int i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, q, i, j, k0, nk, o)) return;
    const long sy = row_stride(q.n), sz = plane_stride(q.n);
    const double *__restrict__ uu = fp(u, q);
    double *__restrict__ ff = fp(F, q);
    const double *__restrict__ fn = fp(Fn1, q);
    const double *__restrict__ in = fp(In, q);
    double *__restrict__ bb = fp(b, q);
    const double ih2 = (double)(q.n + 1) * (double)(q.n + 1);
    const double cc = q.par(c), dl = q.par(delta);
    // every load unguarded (a short column repeats its last plane; without
    // t1 the difference reads u twice and is not added)
    const bool ht = t1.p != nullptr;
    const double *__restrict__ a1 = ht ? fp(t1, q) : uu;
    const double *__restrict__ a0 = ht ? fp(t0, q) : uu;
    double col[KZ + 2], xs[KZ], ys[KZ], rv[KZ], fv[KZ], iv[KZ], x1[KZ], x0[KZ];
#pragma unroll
    for (int w = 0; w < KZ + 2; ++w) col[w] = uu[o + (long)(min(w, nk + 1) - 1) * sz];
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        const long ow = o + (long)min(w, nk - 1) * sz;
        xs[w] = uu[ow - 1] + uu[ow + 1];
        ys[w] = uu[ow - sy] + uu[ow + sy];
        fv[w] = fn[ow];
        iv[w] = in[ow];
        x1[w] = a1[ow];
        x0[w] = a0[ow];
    }
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        double v = col[w + 1] - dl * fv[w] + iv[w];
        if (ht) v = v + (x1[w] - x0[w]);
        rv[w] = v;
    }
#pragma unroll
    for (int w = 0; w < KZ; ++w) {
        if (w < nk) {
            double s = xs[w];
            s += ys[w] + (col[w] + col[w + 2]);
            s -= 6.0 * col[w + 1];
            ff[o + (long)w * sz] = cc * (ih2 * s);
            bb[o + (long)w * sz] = rv[w];
        }
    }
}

struct IntMap {
    int v[MAXN];
};

// Launched on the coarse grids (q.n = coarse n, fine n = 2 (nc + 1) - 1).
template <int DIM, int NNF, int NNC>
__global__ __launch_bounds__(BLOCK) void fas_inject_kernel(Tiling t, int nnf_rt, int nnc_rt, IntMap cmap, double dt,
                                                           const double *__restrict__ Qf, View<double> Uf,
                                                           View<double> Ff, View<double> Uc,
                                                           View<double> Uold, View<double> Tau, View<double> Tauf)
{
    const int nnf = NNF > 0 ? NNF : nnf_rt, nnc = NNC > 0 ? NNC : nnc_rt;
    Pt q; int I, J, K; long o;
    if (!tile_point<DIM>(t, q, I, J, K, o)) return;
    const int nf = 2 * (q.n + 1) - 1;
    const long f_node = node_stride(nf, DIM), c_node = node_stride(q.n, DIM);
    const double h = q.par(dt);
    const long fo = DIM == 3 ? 2L * I + 2L * J * row_stride(nf) + 2L * K * plane_stride(nf) : 2L * I;
    const double *uf = fp(Uf, q) + fo;
    const double *ff = fp(Ff, q) + fo;
    // every load before the first store (the finer tau read from F when
    // absent, unused)
    double fv[MAXN], uv[MAXN], tv[MAXN];
    for (int w = 0; w < nnf; ++w) fv[w] = ff[w * f_node];
    double *uc = fp(Uc, q) + o, *uo = fp(Uold, q) + o, *ta = fp(Tau, q) + o;
    const bool htf = Tauf.p != nullptr;
    const double *tf = htf ? fp(Tauf, q) + fo : ff;
    for (int mc = 0; mc < nnc; ++mc) {
        const int mf = cmap.v[mc];
        uv[mc] = uf[mf * f_node];
        tv[mc] = tf[mf * f_node];
    }
    for (int mc = 0; mc < nnc; ++mc) {
        const int mf = cmap.v[mc];
        uc[mc * c_node] = uv[mc];
        uo[mc * c_node] = uv[mc];
        double acc = 0.0;
        for (int w = 0; w < nnf; ++w) acc += Qf[mf * nnf + w] * fv[w];
        ta[mc * c_node] = htf ? h * acc + tv[mc] : h * acc;
    }
}

template <int DIM, int NNC>
__global__ __launch_bounds__(BLOCK) void fas_tau_kernel(Tiling t, int nnc_rt, double dt, const double *__restrict__ Qc,
                                                        View<double> Fc, View<double> Tau)
{
    const int nnc = NNC > 0 ? NNC : nnc_rt;
    Pt q; int I, J, K; long o;
    if (!tile_point<DIM>(t, q, I, J, K, o)) return;
    const long c_node = node_stride(q.n, DIM);
    const double h = q.par(dt);
    const double *fc = fp(Fc, q) + o;
    double fv[MAXN];
    for (int w = 0; w < nnc; ++w) fv[w] = fc[w * c_node];
    double *ta = fp(Tau, q) + o;
    for (int mc = 0; mc < nnc; ++mc) {
        double acc = 0.0;
        for (int w = 0; w < nnc; ++w) acc += Qc[mc * nnc + w] * fv[w];
        ta[mc * c_node] = ta[mc * c_node] - h * acc;
    }
}

template <int DIM, int NNF, int NNC>
__global__ __launch_bounds__(BLOCK) void interp_coarse_kernel(Tiling t, int nnf_rt, int nnc_rt, const double *__restrict__ Lt,
                                                              View<double> Uc, View<double> Uold, View<double> DC)
{
    const int nnf = NNF > 0 ? NNF : nnf_rt, nnc = NNC > 0 ? NNC : nnc_rt;
    Pt q; int I, J, K; long o;
    if (!tile_point<DIM>(t, q, I, J, K, o)) return;
    const long c_node = node_stride(q.n, DIM), dc_node = c_node;
    const double *uc = fp(Uc, q) + o, *uo = fp(Uold, q) + o;
    double d[MAXN];
    for (int mc = 0; mc < nnc; ++mc) d[mc] = uc[mc * c_node] - uo[mc * c_node];
    double *dc = fp(DC, q) + o;
    for (int m = 0; m < nnf; ++m) {
        double acc = 0.0;
        for (int mc = 0; mc < nnc; ++mc) acc += Lt[m * nnc + mc] * d[mc];
        dc[m * dc_node] = acc;
    }
}

__device__ inline unsigned long long abs_bits(double x)
{
    return (unsigned long long)__double_as_longlong(fabs(x));
}

__device__ inline unsigned long long wave_max(unsigned long long v)
{
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Fields are (problem, slice) pairs, P slices per problem, slice fastest.
// U0 = the problem's block initial value for slice 0, else U[item-1][nn-1].
template <int DIM, int NN>
__global__ __launch_bounds__(BLOCK) void colloc_resid_kernel(Tiling t, int nn_rt, int P, int first, double dt,
                                                             const double *__restrict__ Q, View<double> U,
                                                             View<double> F, View<double> ublock,
                                                             unsigned long long *res_bits,
                                                             unsigned long long *u0_bits)
{
    const int nn = NN > 0 ? NN : nn_rt;
    Pt q; int i, j, k; long o;
    const bool ok = tile_point<DIM>(t, q, i, j, k, o);
    unsigned long long rm = 0, um = 0;
    if (ok) {
        const long node = node_stride(q.n, DIM);
        const double h = q.par(dt);
        double u0;
        if ((first + q.item) % P == 0) {
            Pt qp = q;
            qp.item = (first + q.item) / P;
            u0 = fp(ublock, qp)[o];
        } else {
            Pt qm = q;
            qm.item = q.item - 1;
            u0 = fp(U, qm)[o + (nn - 1) * node];
        }
        const double *uu = fp(U, q) + o, *ff = fp(F, q) + o;
        double fv[MAXN];
        for (int w = 0; w < nn; ++w) fv[w] = ff[w * node];
        for (int m = 0; m < nn; ++m) {
            double acc = 0.0;
            for (int w = 0; w < nn; ++w) acc += Q[m * nn + w] * fv[w];
            const unsigned long long r = abs_bits(u0 - uu[m * node] + h * acc);
            rm = r > rm ? r : rm;
        }
        um = abs_bits(u0);
    }
    Pt qb;
    if (!tile_block_item<DIM>(t, qb)) return;
    int flat = qb.item;
    for (int s = 0; s < qb.sg; ++s) flat += t.seg_count(s);
    rm = wave_max(rm);
    um = wave_max(um);
    __shared__ unsigned long long part[2][BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { part[0][wv] = rm; part[1][wv] = um; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = part[0][0], b = part[1][0];
        for (int w = 1; w < BLOCK / 64; ++w) {
            a = part[0][w] > a ? part[0][w] : a;
            b = part[1][w] > b ? part[1][w] : b;
        }
        const int slot = (int)(blockIdx.x % (unsigned)k::RSLOTS);
        if (a) atomicMax(res_bits + (long)flat * k::RSLOTS + slot, a);
        if (b) atomicMax(u0_bits + (long)flat * k::RSLOTS + slot, b);
    }
}

// Launched on the coarse grids.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void inject_kernel(Tiling t, View<double> uf, View<double> uc)
{
    Pt q; int I, J, K; long o;
    if (!tile_point<DIM>(t, q, I, J, K, o)) return;
    const int nf = 2 * (q.n + 1) - 1;
    const long fo = DIM == 3 ? 2L * I + 2L * J * row_stride(nf) + 2L * K * plane_stride(nf) : 2L * I;
    fp(uc, q)[o] = fp(uf, q)[fo];
}

// dense[item][z][y][x] <-> field; single-segment launches.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void pack_kernel(Tiling t, View<double> f, double *dense)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const long n = q.n;
    const long d = DIM == 3 ? (i - 1) + n * ((j - 1) + n * (long)(k - 1)) : i - 1;
    dense[(long)q.item * interior_points(q.n, DIM) + d] = fp(f, q)[o];
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void unpack_kernel(Tiling t, const double *dense, View<double> f)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const long n = q.n;
    const long d = DIM == 3 ? (i - 1) + n * ((j - 1) + n * (long)(k - 1)) : i - 1;
    fp(f, q)[o] = dense[(long)q.item * interior_points(q.n, DIM) + d];
}

inline dim3 grid_of(const Tiling &t) { return dim3((unsigned)grid_blocks(t)); }

#define PFMG_DISPATCH(t, KER, ...)                                                          \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                 \
        else KER<1><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                              \
        return hipGetLastError();                                                           \
    } while (0)

#define PFMG_DISPATCH_N(t, KER, NN, ...)                                                    \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3, NN><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);             \
        else KER<1, NN><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                          \
        return hipGetLastError();                                                           \
    } while (0)

#define PFMG_DISPATCH_N2(t, KER, NA, NB, ...)                                               \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3, NA, NB><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);         \
        else KER<1, NA, NB><<<grid_of(t), BLOCK, 0, s>>>(__VA_ARGS__);                      \
        return hipGetLastError();                                                           \
    } while (0)

}  // namespace

namespace k {

hipError_t apply_L(const Tiling &t, double nu, View<double> u, View<double> F, hipStream_t s)
{
    if (stencil_z_ok(t)) return apply_L_z(t, nu, u, F, s);
    if (t.dim == 3 && grid_blocks(t) > 0) {
        apply_L_kz_kernel<<<(unsigned)col_blocks<KZ>(t), BLOCK, 0, s>>>(t, nu, u, F);
        return hipGetLastError();
    }
    PFMG_DISPATCH(t, apply_L_kernel, t, nu, u, F);
}

hipError_t sdc_integrals(const Tiling &t, int nn, double dt, const double *S, View<double> F, View<double> I,
                         hipStream_t s)
{
    if (nn > MAXN) return hipErrorInvalidValue;
    if (nn == 5) PFMG_DISPATCH_N(t, sdc_integrals_kernel, 5, t, nn, dt, S, F, I);
    if (nn == 3) PFMG_DISPATCH_N(t, sdc_integrals_kernel, 3, t, nn, dt, S, F, I);
    PFMG_DISPATCH_N(t, sdc_integrals_kernel, 0, t, nn, dt, S, F, I);
}

hipError_t sdc_start(const Tiling &t, int nn, double dt, const double *S, double delta1, View<double> U,
                     View<double> F, View<double> Usrc, View<double> Fsrc, View<double> I, View<double> tau,
                     View<double> b, hipStream_t s, double nu0)
{
    if (nn < 2 || nn > MAXN || (Usrc.p != nullptr) != (Fsrc.p != nullptr)) return hipErrorInvalidValue;
    if (nn == 5) PFMG_DISPATCH_N(t, sdc_start_kernel, 5, t, nn, dt, S, delta1, U, F, Usrc, Fsrc, I, tau, b, nu0);
    if (nn == 3) PFMG_DISPATCH_N(t, sdc_start_kernel, 3, t, nn, dt, S, delta1, U, F, Usrc, Fsrc, I, tau, b, nu0);
    PFMG_DISPATCH_N(t, sdc_start_kernel, 0, t, nn, dt, S, delta1, U, F, Usrc, Fsrc, I, tau, b, nu0);
}

hipError_t solve_F_rhs(const Tiling &t, double delta, View<double> U, View<double> B, View<double> F,
                       double delta_next, View<double> Fn1, View<double> In, View<double> t1, View<double> t0,
                       hipStream_t s)
{
    if ((Fn1.p != nullptr) != (In.p != nullptr) || (t1.p != nullptr) != (t0.p != nullptr)) return hipErrorInvalidValue;
    PFMG_DISPATCH(t, solve_F_rhs_kernel, t, delta, U, B, F, delta_next, Fn1, In, t1, t0);
}

bool apply_L_rhs_ok(const Tiling &t) { return t.dim == 3 && !stencil_z_ok(t); }

hipError_t apply_L_rhs(const Tiling &t, double nu, View<double> u, View<double> F, double delta, View<double> Fn1,
                       View<double> In, View<double> t1, View<double> t0, View<double> b, hipStream_t s)
{
    if (!apply_L_rhs_ok(t) || (t1.p != nullptr) != (t0.p != nullptr)) return hipErrorInvalidValue;
    if (grid_blocks(t) == 0) return hipSuccess;
    apply_L_rhs_kz_kernel<<<(unsigned)col_blocks<KZ>(t), BLOCK, 0, s>>>(t, nu, u, F, delta, Fn1, In, t1, t0, b);
    return hipGetLastError();
}

hipError_t sdc_rhs(const Tiling &t, double delta, View<double> Um, View<double> Fm1, View<double> Im,
                   View<double> tau1, View<double> tau0, View<double> b, hipStream_t s)
{
    PFMG_DISPATCH(t, sdc_rhs_kernel, t, delta, Um, Fm1, Im, tau1, tau0, b);
}

hipError_t fas_inject(const Tiling &t, int nnf, int nnc, const int *cmap, double dt, const double *Qf,
                      View<double> Uf, View<double> Ff, View<double> Uc, View<double> Uold, View<double> Tau,
                      hipStream_t s, View<double> Tauf)
{
    if (nnf > MAXN || nnc > MAXN) return hipErrorInvalidValue;
    IntMap m{};
    for (int w = 0; w < nnc; ++w) m.v[w] = cmap[w];
    if (nnf == 5 && nnc == 3)
        PFMG_DISPATCH_N2(t, fas_inject_kernel, 5, 3, t, nnf, nnc, m, dt, Qf, Uf, Ff, Uc, Uold, Tau, Tauf);
    PFMG_DISPATCH_N2(t, fas_inject_kernel, 0, 0, t, nnf, nnc, m, dt, Qf, Uf, Ff, Uc, Uold, Tau, Tauf);
}

hipError_t fas_tau(const Tiling &t, int nnc, double dt, const double *Qc, View<double> Fc, View<double> Tau,
                   hipStream_t s)
{
    if (nnc > MAXN) return hipErrorInvalidValue;
    if (nnc == 3) PFMG_DISPATCH_N(t, fas_tau_kernel, 3, t, nnc, dt, Qc, Fc, Tau);
    PFMG_DISPATCH_N(t, fas_tau_kernel, 0, t, nnc, dt, Qc, Fc, Tau);
}

hipError_t interp_coarse(const Tiling &t, int nnf, int nnc, const double *Lt, View<double> Uc,
                         View<double> Uold, View<double> DC, hipStream_t s)
{
    if (nnf > MAXN || nnc > MAXN) return hipErrorInvalidValue;
    if (nnf == 5 && nnc == 3) PFMG_DISPATCH_N2(t, interp_coarse_kernel, 5, 3, t, nnf, nnc, Lt, Uc, Uold, DC);
    PFMG_DISPATCH_N2(t, interp_coarse_kernel, 0, 0, t, nnf, nnc, Lt, Uc, Uold, DC);
}

hipError_t colloc_resid(const Tiling &t, int nn, int P, double dt, const double *Q, View<double> U,
                        View<double> F, View<double> ublock, unsigned long long *res_bits,
                        unsigned long long *u0_bits, hipStream_t s, int first)
{
    if (nn > MAXN || P < 1 || first < 0) return hipErrorInvalidValue;
    if (nn == 5)
        PFMG_DISPATCH_N(t, colloc_resid_kernel, 5, t, nn, P, first, dt, Q, U, F, ublock, res_bits, u0_bits);
    PFMG_DISPATCH_N(t, colloc_resid_kernel, 0, t, nn, P, first, dt, Q, U, F, ublock, res_bits, u0_bits);
}

hipError_t inject(const Tiling &t, View<double> uf, View<double> uc, hipStream_t s)
{
    PFMG_DISPATCH(t, inject_kernel, t, uf, uc);
}

hipError_t pack(const Tiling &t, View<double> f, double *dense, hipStream_t s)
{
    PFMG_DISPATCH(t, pack_kernel, t, f, dense);
}

hipError_t unpack(const Tiling &t, const double *dense, View<double> f, hipStream_t s)
{
    PFMG_DISPATCH(t, unpack_kernel, t, dense, f);
}

}  // namespace k
}  // namespace pfmg
