// SDC, FAS and collocation-residual kernels on gfx950 (FP64).
//
//  apply_L       F = nu L_h u, the right-hand side of the semi-discrete
//                heat equation at one node (Sec. 4.1 / 4.2).
//  sdc_integrals I_m = dt sum_i (q_{m+1,i} - q_{m,i}) F_i (eq. sdc-be),
//                all M node-to-node integrals of one slice in one pass.
//  sdc_rhs       right-hand side of the node solve of eq. SDCcompactLIII in
//                node-to-node form, plus the FAS difference on level 1.
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

template <typename T>
__device__ inline T *fp(View<T> v, int item) { return v.p + (long)item * v.stride; }

template <int DIM>
__global__ __launch_bounds__(BLOCK) void apply_L_kernel(Tiling t, double c, View<double> u, View<double> F)
{
    int item, i, j, k; long o;
    if (!tile_point<DIM>(t, item, i, j, k, o)) return;
    const double *uu = fp(u, item);
    const double ih2 = (double)(t.n + 1) * (double)(t.n + 1);
    fp(F, item)[o] = c * (ih2 * d2sum<DIM>(uu, o, row_stride(t.n), plane_stride(t.n)));
}

// Column-blocked 3D variant (KZ planes per thread, loads before stores).
constexpr int KZ = 4;
__global__ __launch_bounds__(BLOCK) void apply_L_kz_kernel(Tiling t, double c, View<double> u, View<double> F)
{
    int item, i, j, k0, nk; long o;
    if (!tile_col<KZ>(t, item, i, j, k0, nk, o)) return;
    const long sy = row_stride(t.n), sz = plane_stride(t.n);
    const double *__restrict__ uu = fp(u, item);
    double *__restrict__ ff = fp(F, item);
    const double ih2 = (double)(t.n + 1) * (double)(t.n + 1);
    double col[KZ + 2], xs[KZ], ys[KZ];
#pragma unroll
    for (int q = 0; q < KZ + 2; ++q) col[q] = q <= nk + 1 ? uu[o + (long)(q - 1) * sz] : 0.0;
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        if (q < nk) {
            const long cc = o + (long)q * sz;
            xs[q] = uu[cc - 1] + uu[cc + 1];
            ys[q] = uu[cc - sy] + uu[cc + sy];
        }
    }
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        if (q < nk) {
            double s = xs[q];
            s += ys[q] + (col[q] + col[q + 2]);
            s -= 6.0 * col[q + 1];
            ff[o + (long)q * sz] = c * (ih2 * s);
        }
    }
}

// NN > 0 fixes the node count at compile time (node values stay in
// registers); NN == 0 is the generic path for any count up to MAXN.
template <int DIM, int NN>
__global__ __launch_bounds__(BLOCK) void sdc_integrals_kernel(Tiling t, int nn_rt, double dt, const double *__restrict__ S,
                                                              View<double> F, long f_node, View<double> I, long i_node)
{
    const int nn = NN > 0 ? NN : nn_rt;
    int item, i, j, k; long o;
    if (!tile_point<DIM>(t, item, i, j, k, o)) return;
    const double *f = fp(F, item) + o;
    double fv[MAXN];
    for (int q = 0; q < nn; ++q) fv[q] = f[q * f_node];
    double *out = fp(I, item) + o;
    for (int m = 0; m + 1 < nn; ++m) {
        double acc = 0.0;
        for (int q = 0; q < nn; ++q) acc += S[m * nn + q] * fv[q];
        out[m * i_node] = dt * acc;
    }
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void sdc_rhs_kernel(Tiling t, double delta, View<double> Um, View<double> Fm1,
                                                        View<double> Im, View<double> t1, View<double> t0, View<double> b)
{
    int item, i, j, k; long o;
    if (!tile_point<DIM>(t, item, i, j, k, o)) return;
    double v = fp(Um, item)[o] - delta * fp(Fm1, item)[o] + fp(Im, item)[o];
    if (t1.p) v = v + (fp(t1, item)[o] - fp(t0, item)[o]);
    fp(b, item)[o] = v;
}

struct IntMap {
    int v[MAXN];
};

// t.n = coarse n.
template <int DIM, int NNF, int NNC>
__global__ __launch_bounds__(BLOCK) void fas_inject_kernel(Tiling t, int nf, int nnf_rt, int nnc_rt, IntMap cmap, double dt,
                                                           const double *__restrict__ Qf, View<double> Uf,
                                                           View<double> Ff, long f_node, View<double> Uc,
                                                           View<double> Uold, View<double> Tau, long c_node)
{
    const int nnf = NNF > 0 ? NNF : nnf_rt, nnc = NNC > 0 ? NNC : nnc_rt;
    int item, I, J, K; long o;
    if (!tile_point<DIM>(t, item, I, J, K, o)) return;
    const long fo = DIM == 3 ? 2L * I + 2L * J * row_stride(nf) + 2L * K * plane_stride(nf) : 2L * I;
    const double *uf = fp(Uf, item) + fo;
    const double *ff = fp(Ff, item) + fo;
    double fv[MAXN];
    for (int q = 0; q < nnf; ++q) fv[q] = ff[q * f_node];
    double *uc = fp(Uc, item) + o, *uo = fp(Uold, item) + o, *ta = fp(Tau, item) + o;
    for (int mc = 0; mc < nnc; ++mc) {
        const int mf = cmap.v[mc];
        const double v = uf[mf * f_node];
        uc[mc * c_node] = v;
        uo[mc * c_node] = v;
        double acc = 0.0;
        for (int q = 0; q < nnf; ++q) acc += Qf[mf * nnf + q] * fv[q];
        ta[mc * c_node] = dt * acc;
    }
}

template <int DIM, int NNC>
__global__ __launch_bounds__(BLOCK) void fas_tau_kernel(Tiling t, int nnc_rt, double dt, const double *__restrict__ Qc,
                                                        View<double> Fc, View<double> Tau, long c_node)
{
    const int nnc = NNC > 0 ? NNC : nnc_rt;
    int item, I, J, K; long o;
    if (!tile_point<DIM>(t, item, I, J, K, o)) return;
    const double *fc = fp(Fc, item) + o;
    double fv[MAXN];
    for (int q = 0; q < nnc; ++q) fv[q] = fc[q * c_node];
    double *ta = fp(Tau, item) + o;
    for (int mc = 0; mc < nnc; ++mc) {
        double acc = 0.0;
        for (int q = 0; q < nnc; ++q) acc += Qc[mc * nnc + q] * fv[q];
        ta[mc * c_node] = ta[mc * c_node] - dt * acc;
    }
}

template <int DIM, int NNF, int NNC>
__global__ __launch_bounds__(BLOCK) void interp_coarse_kernel(Tiling t, int nnf_rt, int nnc_rt, const double *__restrict__ Lt,
                                                              View<double> Uc, View<double> Uold, long c_node,
                                                              View<double> DC, long dc_node)
{
    const int nnf = NNF > 0 ? NNF : nnf_rt, nnc = NNC > 0 ? NNC : nnc_rt;
    int item, I, J, K; long o;
    if (!tile_point<DIM>(t, item, I, J, K, o)) return;
    const double *uc = fp(Uc, item) + o, *uo = fp(Uold, item) + o;
    double d[MAXN];
    for (int mc = 0; mc < nnc; ++mc) d[mc] = uc[mc * c_node] - uo[mc * c_node];
    double *dc = fp(DC, item) + o;
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

// item = slice p; U0 = ublock for p = 0, else U[p-1][nn-1].
template <int DIM, int NN>
__global__ __launch_bounds__(BLOCK) void colloc_resid_kernel(Tiling t, int nn_rt, double dt, const double *__restrict__ Q,
                                                             View<double> U, View<double> F, long node,
                                                             const double *__restrict__ ublock,
                                                             unsigned long long *res_bits,
                                                             unsigned long long *u0_bits)
{
    const int nn = NN > 0 ? NN : nn_rt;
    int item, i, j, k; long o;
    const bool ok = tile_point<DIM>(t, item, i, j, k, o);
    unsigned long long rm = 0, um = 0;
    if (ok) {
        const double u0 = item == 0 ? ublock[o] : fp(U, item - 1)[o + (nn - 1) * node];
        const double *uu = fp(U, item) + o, *ff = fp(F, item) + o;
        double fv[MAXN];
        for (int q = 0; q < nn; ++q) fv[q] = ff[q * node];
        for (int m = 0; m < nn; ++m) {
            double acc = 0.0;
            for (int q = 0; q < nn; ++q) acc += Q[m * nn + q] * fv[q];
            const unsigned long long r = abs_bits(u0 - uu[m * node] + dt * acc);
            rm = r > rm ? r : rm;
        }
        um = abs_bits(u0);
    }
    const unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    const int blk_item = (int)(bid / tiles_per_field(t.n, DIM));
    if (blk_item >= t.count) return;
    rm = wave_max(rm);
    um = wave_max(um);
    __shared__ unsigned long long part[2][BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { part[0][wv] = rm; part[1][wv] = um; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = part[0][0], b = part[1][0];
        for (int q = 1; q < BLOCK / 64; ++q) {
            a = part[0][q] > a ? part[0][q] : a;
            b = part[1][q] > b ? part[1][q] : b;
        }
        const int slot = (int)(bid % (unsigned)k::RSLOTS);
        if (a) atomicMax(res_bits + (long)blk_item * k::RSLOTS + slot, a);
        if (b) atomicMax(u0_bits + (long)blk_item * k::RSLOTS + slot, b);
    }
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void inject_kernel(Tiling t, int nf, View<double> uf, View<double> uc)
{
    int item, I, J, K; long o;
    if (!tile_point<DIM>(t, item, I, J, K, o)) return;
    const long fo = DIM == 3 ? 2L * I + 2L * J * row_stride(nf) + 2L * K * plane_stride(nf) : 2L * I;
    fp(uc, item)[o] = fp(uf, item)[fo];
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void pack_kernel(Tiling t, View<double> f, double *dense)
{
    int item, i, j, k; long o;
    if (!tile_point<DIM>(t, item, i, j, k, o)) return;
    const long n = t.n;
    const long d = DIM == 3 ? (i - 1) + n * ((j - 1) + n * (long)(k - 1)) : i - 1;
    dense[(long)item * interior_points(t.n, DIM) + d] = fp(f, item)[o];
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void unpack_kernel(Tiling t, const double *dense, View<double> f)
{
    int item, i, j, k; long o;
    if (!tile_point<DIM>(t, item, i, j, k, o)) return;
    const long n = t.n;
    const long d = DIM == 3 ? (i - 1) + n * ((j - 1) + n * (long)(k - 1)) : i - 1;
    fp(f, item)[o] = dense[(long)item * interior_points(t.n, DIM) + d];
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
    if (t.dim == 3 && grid_blocks(t) > 0) {
        apply_L_kz_kernel<<<(unsigned)(col_tiles_per_field(t.n, KZ) * t.count), BLOCK, 0, s>>>(t, nu, u, F);
        return hipGetLastError();
    }
    PFMG_DISPATCH(t, apply_L_kernel, t, nu, u, F);
}

hipError_t sdc_integrals(const Tiling &t, int nn, double dt, const double *S, View<double> F, long f_node,
                         View<double> I, long i_node, hipStream_t s)
{
    if (nn > MAXN) return hipErrorInvalidValue;
    if (nn == 5) PFMG_DISPATCH_N(t, sdc_integrals_kernel, 5, t, nn, dt, S, F, f_node, I, i_node);
    if (nn == 3) PFMG_DISPATCH_N(t, sdc_integrals_kernel, 3, t, nn, dt, S, F, f_node, I, i_node);
    PFMG_DISPATCH_N(t, sdc_integrals_kernel, 0, t, nn, dt, S, F, f_node, I, i_node);
}

hipError_t sdc_rhs(const Tiling &t, double delta, View<double> Um, View<double> Fm1, View<double> Im,
                   View<double> tau1, View<double> tau0, View<double> b, hipStream_t s)
{
    PFMG_DISPATCH(t, sdc_rhs_kernel, t, delta, Um, Fm1, Im, tau1, tau0, b);
}

hipError_t fas_inject(const Tiling &t, int nf, int nnf, int nnc, const int *cmap, double dt, const double *Qf,
                      View<double> Uf, View<double> Ff, long f_node, View<double> Uc, View<double> Uold,
                      View<double> Tau, long c_node, hipStream_t s)
{
    if (nnf > MAXN || nnc > MAXN) return hipErrorInvalidValue;
    IntMap m{};
    for (int q = 0; q < nnc; ++q) m.v[q] = cmap[q];
    if (nnf == 5 && nnc == 3)
        PFMG_DISPATCH_N2(t, fas_inject_kernel, 5, 3, t, nf, nnf, nnc, m, dt, Qf, Uf, Ff, f_node, Uc, Uold, Tau, c_node);
    PFMG_DISPATCH_N2(t, fas_inject_kernel, 0, 0, t, nf, nnf, nnc, m, dt, Qf, Uf, Ff, f_node, Uc, Uold, Tau, c_node);
}

hipError_t fas_tau(const Tiling &t, int nnc, double dt, const double *Qc, View<double> Fc, View<double> Tau,
                   long c_node, hipStream_t s)
{
    if (nnc > MAXN) return hipErrorInvalidValue;
    if (nnc == 3) PFMG_DISPATCH_N(t, fas_tau_kernel, 3, t, nnc, dt, Qc, Fc, Tau, c_node);
    PFMG_DISPATCH_N(t, fas_tau_kernel, 0, t, nnc, dt, Qc, Fc, Tau, c_node);
}

hipError_t interp_coarse(const Tiling &t, int nnf, int nnc, const double *Lt, View<double> Uc,
                         View<double> Uold, long c_node, View<double> DC, long dc_node, hipStream_t s)
{
    if (nnf > MAXN || nnc > MAXN) return hipErrorInvalidValue;
    if (nnf == 5 && nnc == 3)
        PFMG_DISPATCH_N2(t, interp_coarse_kernel, 5, 3, t, nnf, nnc, Lt, Uc, Uold, c_node, DC, dc_node);
    PFMG_DISPATCH_N2(t, interp_coarse_kernel, 0, 0, t, nnf, nnc, Lt, Uc, Uold, c_node, DC, dc_node);
}

hipError_t colloc_resid(const Tiling &t, int nn, double dt, const double *Q, View<double> U, View<double> F,
                        long node, const double *ublock, unsigned long long *res_bits,
                        unsigned long long *u0_bits, hipStream_t s)
{
    if (nn > MAXN) return hipErrorInvalidValue;
    if (nn == 5) PFMG_DISPATCH_N(t, colloc_resid_kernel, 5, t, nn, dt, Q, U, F, node, ublock, res_bits, u0_bits);
    PFMG_DISPATCH_N(t, colloc_resid_kernel, 0, t, nn, dt, Q, U, F, node, ublock, res_bits, u0_bits);
}

hipError_t inject(const Tiling &t, int nf, View<double> uf, View<double> uc, hipStream_t s)
{
    PFMG_DISPATCH(t, inject_kernel, t, nf, uf, uc);
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
