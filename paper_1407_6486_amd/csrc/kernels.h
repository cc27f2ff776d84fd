// Host-side launchers of the gfx950 kernels.  Every launcher enqueues one
// kernel on `s` and returns the launch status.  Views follow layout.h.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.h"
#include "tile.h"

namespace pfmg {
namespace k {

// ---------------------------------------------------------------- grid ops
// r = b - (I - alpha L_h) u
template <typename T>
hipError_t resid(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> r, hipStream_t s);
// FP64 residual rounded once to FP32 (refinement step of the mixed form)
hipError_t resid_round(const Tiling &t, double alpha, View<double> b, View<double> u,
                       View<float> r32, hipStream_t s);
// out = u + omega (b - H u) / diag(H)
template <typename T>
hipError_t jacobi(const Tiling &t, double alpha, double omega, View<T> b, View<T> u,
                  View<T> out, hipStream_t s);
// First Jacobi sweep from u = 0: out = omega b / diag(H)
template <typename T>
hipError_t jacobi_zero(const Tiling &t, double alpha, double omega, View<T> b, View<T> out,
                       hipStream_t s);
// Red (colour 0: 1-based i+j+k even) or black points, in place.
template <typename T>
hipError_t rbgs(const Tiling &t, double alpha, double omega, int colour, View<T> b, View<T> u,
                hipStream_t s);
// Launch shape of the fused sweep: rows per workgroup, planes per z-chunk.
struct FusedShape {
    int ty, zchunk;
    long blocks;
    size_t lds;
    int nt = 256;   // threads per workgroup: 256 or 512
};
FusedShape rbgs_fused_shape(const Tiling &t, size_t elem, int ty = 0, int target_blocks = 0, int nt = 256);
// Whether the one-pass kernel is instantiated for ty rows per workgroup
// on grids up to nmax points a side with nt (256 or 512) threads.
bool rbgs_fused_ty_ok(int nmax, int ty, int nt);
// One whole red-black sweep out of place (3D, 31 <= n <= 255): uout =
// RBGS(uin); zero_in treats uin as 0 (first sweep of a coarse correction).
// shape: a shape from rbgs_fused_shape for this tiling (nullptr: default).
template <typename T>
hipError_t rbgs_fused(const Tiling &t, double alpha, double omega, bool zero_in, View<T> b, View<T> uin,
                      View<T> uout, hipStream_t s, const FusedShape *shape = nullptr);
// Red pass from u = 0: red points omega b / diag(H), black points 0.
template <typename T>
hipError_t rbgs_zero_red(const Tiling &t, double alpha, double omega, View<T> b, View<T> u,
                         hipStream_t s);
// Whole V(nu1, nu2)-cycle from grid t.n down in LDS, one workgroup per field
// (small grids).  zero_init starts from u = 0 instead of reading u.
// LDS the kernel may take per workgroup on the current device (the device's
// per-workgroup limit less the kernel's static level table); a grid whose
// vcycle_bottom_lds exceeds it takes the per-level path.
size_t bottom_lds_max();
size_t vcycle_bottom_lds(int n0, int dim, int smoother, size_t elem);
template <typename T>
hipError_t vcycle_bottom(const Tiling &t, double alpha, int smoother, double omega, int nu1, int nu2, bool zero_init,
                         View<T> b, View<T> u, hipStream_t s);
// One-pass z-marching residual + full weighting (3D, odd fine n in
// [63, 255]); resid_restrict takes it wherever resid_restrict_z_ok holds.
bool resid_restrict_z_ok(const Tiling &t);
template <typename T>
hipError_t resid_restrict_z(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> bc, hipStream_t s);
// Full weighting of a fine array (t.n = fine n) onto the coarse grid.
template <typename T>
hipError_t restrict_fw(const Tiling &t, View<T> r, View<T> bc, hipStream_t s);
// Fused: coarse rhs = FW(b - H u) on the fine grid (t.n = fine n).
template <typename T>
hipError_t resid_restrict(const Tiling &t, double alpha, View<T> b, View<T> u, View<T> bc,
                          hipStream_t s);
// u += P ec, d-linear (t.n = fine n).
template <typename T>
hipError_t prolong_add(const Tiling &t, View<T> ec, View<T> u, hipStream_t s);
// The same in one z-marching pass (3D, odd fine n in [31, 255], launches of
// 2^19 points or more); prolong_add takes it wherever prolong_z_ok holds.
// kch_force > 0 fixes the coarse planes per workgroup.
bool prolong_z_ok(const Tiling &t);
template <typename T>
hipError_t prolong_z(const Tiling &t, View<T> ec, View<T> u, hipStream_t s, int kch_force = 0);
// Exact solve for n in {1, 2}.
template <typename T>
hipError_t coarsest(const Tiling &t, double alpha, View<T> b, View<T> u, hipStream_t s);
template <typename T>
hipError_t zero(const Tiling &t, View<T> u, hipStream_t s);
template <typename T>
hipError_t copy(const Tiling &t, View<T> src, View<T> dst, hipStream_t s);
// u += (double) e
hipError_t add_f32(const Tiling &t, View<float> e, View<double> u, hipStream_t s);
// bits[item] = max(bits[item], |v|_inf as ordered bits); bits must be preset
template <typename T>
hipError_t norm_inf(const Tiling &t, View<T> v, unsigned long long *bits, hipStream_t s);
// bits[item] = max |b - H u|
hipError_t resid_norm(const Tiling &t, double alpha, View<double> b, View<double> u,
                      unsigned long long *bits, hipStream_t s);

// ------------------------------------------------------------ method ops
// F = nu L_h u
hipError_t apply_L(const Tiling &t, double nu, View<double> u, View<double> F, hipStream_t s);
// z-marching F = c L_h u and omega-Jacobi sweep (3D, 31 <= n <= 255, at
// least 2^20 points in the launch; input and output must not overlap);
// apply_L and jacobi take them wherever stencil_z_ok holds.
bool stencil_z_ok(const Tiling &t);
hipError_t apply_L_z(const Tiling &t, double c, View<double> u, View<double> F, hipStream_t s);
template <typename T>
hipError_t jacobi_z(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, View<T> out, hipStream_t s);
// Node stacks: a view's field q points at node 0 of a slice; node m sits
// m slot strides (node_stride of the grid) further.
// I[m] = dt sum_i S[m][i] F[i], m = 0..nn-2, per slice (item = slice).
hipError_t sdc_integrals(const Tiling &t, int nn, double dt, const double *S, View<double> F,
                         View<double> I, hipStream_t s);
// b = U[m] - delta F[m+1] + I[m] (+ tau1 - tau0 when tau1.p != nullptr)
hipError_t sdc_rhs(const Tiling &t, double delta, View<double> Um, View<double> Fm1,
                   View<double> Im, View<double> tau1, View<double> tau0, View<double> b,
                   hipStream_t s);
// sdc_integrals and the first node's sdc_rhs in one pass (node 0 of U and F
// first copied from Usrc / Fsrc when they are set -- with nu0 > 0, F of
// node 0 is instead nu0 L_h of Usrc, the second-order stencil; tau: all
// coarse nodes, or null on the fine level).
hipError_t sdc_start(const Tiling &t, int nn, double dt, const double *S, double delta1, View<double> U,
                     View<double> F, View<double> Usrc, View<double> Fsrc, View<double> I, View<double> tau,
                     View<double> b, hipStream_t s, double nu0 = 0.0);
// F = (U - B) / delta at the node just solved (B: its right-hand side);
// then, when Fn1 is set, B = U - delta_next Fn1 + In (+ t1 - t0), the next
// node's right-hand side.
hipError_t solve_F_rhs(const Tiling &t, double delta, View<double> U, View<double> B, View<double> F,
                       double delta_next, View<double> Fn1, View<double> In, View<double> t1, View<double> t0,
                       hipStream_t s);
// apply_L into F and, from the same loads of u, sdc_rhs of the next node
// (Fn1, In, t1, t0 as sdc_rhs's Fm1, Im, tau1, tau0); for launches that
// apply_L would run column-blocked (3D, below the z-marching size).
bool apply_L_rhs_ok(const Tiling &t);
// Fourth-order fine level (stencil4.hip): F = nu L4 u; r = b - (u - alpha
// L4 u); one smoothing pass for (I - alpha L4), out of place (colour -1:
// weighted Jacobi on every point; 0 / 1: that colour of the red-black JOR
// from src, the other points copied); u += cubic interpolation of e_c
// (coarse grids (n+1)/2 - 1 >= 3).
hipError_t apply_L4(const Tiling &t, double nu, View<double> u, View<double> F, hipStream_t s);
hipError_t resid4(const Tiling &t, double alpha, View<double> b, View<double> u, View<double> r, hipStream_t s);
hipError_t smooth4(const Tiling &t, double alpha, double omega, int colour, View<double> b, View<double> src,
                   View<double> dst, hipStream_t s);
hipError_t prolong4_add(const Tiling &t, View<double> ec, View<double> u, hipStream_t s);
hipError_t prolong4_add2(const Tiling &t, View<double> ec, View<double> u, View<double> ec2, View<double> u2,
                         hipStream_t s);
hipError_t apply_L_rhs(const Tiling &t, double nu, View<double> u, View<double> F, double delta, View<double> Fn1,
                       View<double> In, View<double> t1, View<double> t0, View<double> b, hipStream_t s);
// FAS injection (t on the coarse grids): Uc[mc] = Uold[mc] = Uf[cmap[mc]] at
// 2J, Tau[mc] = dt sum_i Qf[cmap[mc]][i] Ff[i] (+ Tauf[cmap[mc]], the finer
// level's own FAS term, when Tauf is set) at 2J.
hipError_t fas_inject(const Tiling &t, int nnf, int nnc, const int *cmap, double dt,
                      const double *Qf, View<double> Uf, View<double> Ff,
                      View<double> Uc, View<double> Uold, View<double> Tau, hipStream_t s,
                      View<double> Tauf = View<double>{nullptr, 0});
// Tau[mc] -= dt sum_j Qc[mc][j] Fc[j]   (t.n = coarse n)
hipError_t fas_tau(const Tiling &t, int nnc, double dt, const double *Qc, View<double> Fc,
                   View<double> Tau, hipStream_t s);
// DC[m] = sum_mc Lt[m][mc] (Uc[mc] - Uold[mc]), m = 0..nnf-1 (t.n = coarse n)
hipError_t interp_coarse(const Tiling &t, int nnf, int nnc, const double *Lt, View<double> Uc,
                         View<double> Uold, View<double> DC, hipStream_t s);
// Collocation residual (eq. resid) per slice; each slice's maxima go to
// RSLOTS partial slots (res_bits[p * RSLOTS + w]); bits preset to 0.
constexpr int RSLOTS = 64;
// Fields are (problem, slice) pairs with P slices per problem; ublock holds
// one block initial value per problem.  first: the pair index of the
// launch's field 0 (a launch over slices p0 .. p1-1 of one problem passes
// p0 with U, F and the bits offset to slice p0; the field before it is then
// read from U's previous slot).
hipError_t colloc_resid(const Tiling &t, int nn, int P, double dt, const double *Q, View<double> U,
                        View<double> F, View<double> ublock,
                        unsigned long long *res_bits, unsigned long long *u0_bits, hipStream_t s, int first = 0);
// Point-wise injection uc(J) = uf(2J) (t on the coarse grids).
hipError_t inject(const Tiling &t, View<double> uf, View<double> uc, hipStream_t s);
// dense (n^dim, x fastest) <-> field
hipError_t pack(const Tiling &t, View<double> f, double *dense, hipStream_t s);
hipError_t unpack(const Tiling &t, const double *dense, View<double> f, hipStream_t s);
hipError_t fill_u64(unsigned long long *p, unsigned long long v, int count, hipStream_t s);
// dst[0 .. bytes) = src[0 .. bytes) in 16-byte nontemporal loads / stores
// (bytes a multiple of 16, both 16-byte aligned, not overlapping).
hipError_t stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

}  // namespace k
}  // namespace pfmg
