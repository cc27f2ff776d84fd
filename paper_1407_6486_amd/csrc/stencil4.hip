// Fourth-order spatial discretisation on the fine level (the paper's
// fourth-order runs, Sec. 4.3) and fourth-order spatial interpolation of
// the PFASST coarse correction.
//
//  apply_L4     F = c L4 u: per axis (-u_{i-2} + 16 u_{i-1} - 30 u_i
//               + 16 u_{i+1} - u_{i+2}) / (12 h^2).  The halo holds the
//               zero boundary value one step out; two steps out the value
//               is the odd reflection -u_{1} (or -u_{n}), which keeps the
//               sine modes eigenvectors.  The field layout shares halo
//               words between rows, so that value is selected by index,
//               never read.
//  resid4       r = b - (u - alpha L4 u).
//  smooth4      one pass of weighted Jacobi (every point) or of one colour
//               of the red-black JOR: points of the colour are updated from
//               the input field (the stencil reaches same-colour points two
//               steps away), the others copied; out of place.
//  prolong4_add u += P4 e_c: tensor-product cubic Lagrange interpolation
//               (prolong4_add2: two corrections into two fields at once).
//               A fine point on a coarse point takes its value; between
//               coarse points J and J+1 the cubic through J-1 .. J+2,
//               shifted inwards next to the boundary (whose zero value is
//               one of the four points).
//
// Point-per-thread launches (tile.h) for the stencils; these grids are the
// small fine grids of the fourth-order configurations.  The 3D cubic
// interpolation is separable and z-marching (prolong4z_kernel below).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace pfmg {
namespace {

// 12 x (sum over axes of the 5-point fourth difference) at (i, j, k),
// 1-based, element offset o.
template <int DIM>
__device__ inline double d4sum(const double *__restrict__ u, int n, int i, int j, int k, long o, long sy, long sz)
{
    const double c = u[o];
    auto axis = [&](int x, long st) {
        // the address is clamped to the point itself where the value two
        // steps out is the reflection, so every load stays in the field
        const double m2v = u[x >= 2 ? o - 2 * st : o];
        const double p2v = u[x <= n - 1 ? o + 2 * st : o];
        const double m2 = x >= 2 ? m2v : -c;
        const double p2 = x <= n - 1 ? p2v : -c;
        return -m2 + 16.0 * u[o - st] - 30.0 * c + 16.0 * u[o + st] - p2;
    };
    double s = axis(i, 1);
    if (DIM == 3) {
        s += axis(j, sy);
        s += axis(k, sz);
    }
    return s;
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void apply_L4_kernel(Tiling t, double c, View<double> u, View<double> F)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const double ih2 = (double)(q.n + 1) * (double)(q.n + 1);
    const double d = d4sum<DIM>(fp(u, q), q.n, i, j, k, o, row_stride(q.n), plane_stride(q.n));
    fp(F, q)[o] = q.par(c) * (ih2 * (d / 12.0));
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void resid4_kernel(Tiling t, double alpha, View<double> b, View<double> u,
                                                       View<double> r)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const double ah = q.par(alpha) * (double)(q.n + 1) * (double)(q.n + 1);
    const double *uu = fp(u, q);
    const double d = d4sum<DIM>(uu, q.n, i, j, k, o, row_stride(q.n), plane_stride(q.n));
    fp(r, q)[o] = fp(b, q)[o] - (uu[o] - ah * (d / 12.0));
}

// colour < 0: every point (weighted Jacobi); 0 red, 1 black (red: 1-based
// index sum even).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void smooth4_kernel(Tiling t, double alpha, double omega, int colour,
                                                        View<double> b, View<double> src, View<double> dst)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const double *uu = fp(src, q);
    const double uc = uu[o];
    const int sum1 = DIM == 3 ? i + j + k : i;
    double v = uc;
    if (colour < 0 || (sum1 & 1) == colour) {
        const double a = q.par(alpha);
        const double ah = a * (double)(q.n + 1) * (double)(q.n + 1);
        const double diag = 1.0 + 2.5 * DIM * a * (double)(q.n + 1) * (double)(q.n + 1);
        const double d = d4sum<DIM>(uu, q.n, i, j, k, o, row_stride(q.n), plane_stride(q.n));
        const double r = fp(b, q)[o] - (uc - ah * (d / 12.0));
        v = uc + omega * r / diag;
    }
    fp(dst, q)[o] = v;
}

// Cubic Lagrange weights of fine 1-based index x on coarse 1-based
// indices idx (0 and nc+1 are the boundary).  Returns the count (1 or 4).
// A fine point between coarse points sits at their midpoint, so the
// weights are constants: (-1, 9, 9, -1)/16 on J-1 .. J+2, and next to a
// boundary the shifted stencils (5, 15, -5, 1)/16 and (1, -5, 15, 5)/16
// (exact dyadic values of the Lagrange basis at the midpoint).
__device__ inline int cubic_w(int x, int nc, int *idx, double *w)
{
    if ((x & 1) == 0) {
        idx[0] = x / 2;
        w[0] = 1.0;
        return 1;
    }
    const int J = (x - 1) / 2;
    int lo;
    if (J == 0) {
        lo = 0;
        w[0] = 5.0 / 16; w[1] = 15.0 / 16; w[2] = -5.0 / 16; w[3] = 1.0 / 16;
    } else if (J == nc) {
        lo = nc - 2;
        w[0] = 1.0 / 16; w[1] = -5.0 / 16; w[2] = 15.0 / 16; w[3] = 5.0 / 16;
    } else {
        lo = J - 1;
        w[0] = -1.0 / 16; w[1] = 9.0 / 16; w[2] = 9.0 / 16; w[3] = -1.0 / 16;
    }
    for (int a = 0; a < 4; ++a) idx[a] = lo + a;
    return 4;
}

// Launched on the fine grids; ec on the coarse grids nc = (n+1)/2 - 1.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void prolong4_add_kernel(Tiling t, View<double> ec, View<double> u)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const int nc = coarser(q.n);
    const long syc = row_stride(nc), szc = plane_stride(nc);
    const double *e = fp(ec, q);
    int ix[4], iy[4] = {0, 0, 0, 0}, iz[4] = {0, 0, 0, 0};
    double wx[4], wy[4] = {1.0, 0, 0, 0}, wz[4] = {1.0, 0, 0, 0};
    const int cx = cubic_w(i, nc, ix, wx);
    const int cy = DIM == 3 ? cubic_w(j, nc, iy, wy) : 1;
    const int cz = DIM == 3 ? cubic_w(k, nc, iz, wz) : 1;
    double acc = 0.0;
    for (int c = 0; c < cz; ++c)
        for (int b = 0; b < cy; ++b)
            for (int a = 0; a < cx; ++a) {
                const long oc = DIM == 3 ? (long)ix[a] + (long)iy[b] * syc + (long)iz[c] * szc : (long)ix[a];
                acc += wz[c] * wy[b] * wx[a] * e[oc];
            }
    fp(u, q)[o] += acc;
}

// prolong4_add of two corrections at once (U's and F's in PFASST
// interpolation): the same indices and weights, each sum accumulated as in
// prolong4_add_kernel.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void prolong4_add2_kernel(Tiling t, View<double> ec, View<double> u,
                                                              View<double> ec2, View<double> u2)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<DIM>(t, q, i, j, k, o)) return;
    const int nc = coarser(q.n);
    const long syc = row_stride(nc), szc = plane_stride(nc);
    const double *e = fp(ec, q), *e2 = fp(ec2, q);
    int ix[4], iy[4] = {0, 0, 0, 0}, iz[4] = {0, 0, 0, 0};
    double wx[4], wy[4] = {1.0, 0, 0, 0}, wz[4] = {1.0, 0, 0, 0};
    const int cx = cubic_w(i, nc, ix, wx);
    const int cy = DIM == 3 ? cubic_w(j, nc, iy, wy) : 1;
    const int cz = DIM == 3 ? cubic_w(k, nc, iz, wz) : 1;
    double acc = 0.0, acc2 = 0.0;
    for (int c = 0; c < cz; ++c)
        for (int b = 0; b < cy; ++b)
            for (int a = 0; a < cx; ++a) {
                const long oc = DIM == 3 ? (long)ix[a] + (long)iy[b] * syc + (long)iz[c] * szc : (long)ix[a];
                const double w = wz[c] * wy[b] * wx[a];
                acc += w * e[oc];
                acc2 += w * e2[oc];
            }
    fp(u, q)[o] += acc;
    fp(u2, q)[o] += acc2;
}

// Separable cubic prolongation + correction in 3D, marching upwards
// through the coarse planes.  A workgroup owns TY fine rows (all fine x)
// and a chunk of fine planes [k0, k1).  For each coarse plane K it needs
// (the zero boundary planes 0 and nc+1 included; they are zero in memory):
//   1. the coarse rows of the tile (its fine rows' cubic stencils, with
//      the zero boundary rows) go to LDS, every coarse x with its zero
//      boundary words;
//   2. x pass: every coarse row is interpolated to the fine x of each lane
//      into LDS;
//   3. y pass: each thread interpolates its Q fine rows in y into a
//      register window that keeps the last four coarse planes;
//   4. every fine plane of the chunk whose stencil ends at plane K (the
//      even plane 2K and the odd plane 2K-3; plane 1 at K = 3 and plane n
//      at K = nc+1) takes its z combination of the window and is added to
//      u (both corrections at once with NA = 2).
// Each coarse value is read once per tile (plus the stencil rows and
// planes around it), each fine value of u read and written once: 16 + 1
// bytes per fine point and correction in FP64.  The sums are taken x,
// then y, then z (the order a separable evaluation gives).  The coarse
// rows of plane K+1 and the u values of step K's fine planes are loaded
// at the top of step K, so their latency hides behind its two barriers
// and LDS passes.
template <int RLN, int Q, int NA>
__global__ __launch_bounds__(BLOCK) void prolong4z_kernel(Tiling t, int kch, View<double> ec, View<double> u,
                                                          View<double> ec2, View<double> u2)
{
    constexpr int RPP = BLOCK / RLN;      // fine rows per pass of the workgroup
    constexpr int TY = Q * RPP;           // fine rows per tile
    constexpr int RMAX = TY / 2 + 5;      // coarse rows a tile's stencils reach
    constexpr int CXL = RLN / 2 + 2;      // coarse x 0 .. nc+1 (nc+2 <= RLN/2+1)
    constexpr int CPT = (NA * RMAX * CXL + BLOCK - 1) / BLOCK;   // coarse values per thread and plane
    extern __shared__ unsigned char smem_raw[];
    double *C = reinterpret_cast<double *>(smem_raw);   // [NA][RMAX][CXL]
    double *X = C + NA * RMAX * CXL;                     // [NA][RMAX][RLN]

    unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    Pt qs;
    const int *mask;
    if (!find_seg(t, bid, qs, mask, [kch](int nf) {
            return (long)((nf + TY - 1) / TY) * ((nf + kch - 1) / kch);
        }))
        return;
    const int n = qs.n, nc = coarser(n);
    const int ytiles = (n + TY - 1) / TY, zch = (n + kch - 1) / kch;
    const int item = (int)(bid / (unsigned)(ytiles * zch));
    const int rem = (int)(bid - (unsigned)item * (unsigned)(ytiles * zch));
    const int jt = rem / zch, zc = rem - jt * zch;
    if (mask && !mask[item]) return;
    qs.item = item;
    const int j0 = jt * TY + 1, k0 = zc * kch + 1, k1 = min(k0 + kch, n + 1);
    const int lane = (int)(threadIdx.x % RLN), rsub = (int)(threadIdx.x / RLN);
    const int i = lane + 1;
    const int sy = (int)row_stride(n), sz = (int)plane_stride(n);
    const int syc = (int)row_stride(nc), szc = (int)plane_stride(nc);
    const double *E0 = fp(ec, qs), *E1 = NA > 1 ? fp(ec2, qs) : E0;
    double *U0 = fp(u, qs), *U1 = NA > 1 ? fp(u2, qs) : U0;

    // first coarse index and weights of fine index x's stencil; returns
    // the count (1 on a coarse point, else 4)
    auto stencil = [nc](int x, int &lo, double (&w)[4]) -> int {
        if ((x & 1) == 0) {
            lo = x / 2;
            w[0] = 1.0; w[1] = w[2] = w[3] = 0.0;
            return 1;
        }
        const int J = (x - 1) / 2;
        if (J == 0) {
            lo = 0;
            w[0] = 5.0 / 16; w[1] = 15.0 / 16; w[2] = -5.0 / 16; w[3] = 1.0 / 16;
        } else if (J == nc) {
            lo = nc - 2;
            w[0] = 1.0 / 16; w[1] = -5.0 / 16; w[2] = 15.0 / 16; w[3] = 5.0 / 16;
        } else {
            lo = J - 1;
            w[0] = -1.0 / 16; w[1] = 9.0 / 16; w[2] = 9.0 / 16; w[3] = -1.0 / 16;
        }
        return 4;
    };
    // the coarse indices the stencils of fine indices [x0, x1] reach: the
    // lowest comes from one of the first two, the highest from one of the
    // last two (an odd index reaches one further than its even neighbour)
    auto reach = [&](int x0, int x1, int &lo, int &hi) {
        lo = 1 << 30;
        hi = -1;
        for (int x = x0; x <= x1 && x <= x0 + 1; ++x) {
            int l;
            double w[4];
            stencil(x, l, w);
            lo = min(lo, l);
        }
        for (int x = max(x0, x1 - 1); x <= x1; ++x) {
            int l;
            double w[4];
            const int c = stencil(x, l, w);
            hi = max(hi, l + c - 1);
        }
    };
    int Rlo, Rhi, Klo, Khi;
    reach(j0, min(j0 + TY - 1, n), Rlo, Rhi);   // coarse rows of the tile, R <= RMAX
    reach(k0, k1 - 1, Klo, Khi);                // coarse planes of the chunk
    const int R = Rhi - Rlo + 1;

    // this thread's share of a coarse plane's tile: source (relative to
    // the plane) and LDS slot of each value
    const double *csrc[CPT];
    int cdst[CPT];
    const int ctot = NA * R * (nc + 2);
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int e = (int)threadIdx.x + c * BLOCK;
        csrc[c] = nullptr;
        cdst[c] = 0;
        if (e < ctot) {
            const int a = e / (R * (nc + 2));
            const int r2 = e - a * R * (nc + 2);
            const int r = r2 / (nc + 2), x = r2 - r * (nc + 2);
            csrc[c] = (a ? E1 : E0) + x + (Rlo + r) * syc;
            cdst[c] = (a * RMAX + r) * CXL + x;
        }
    }
    auto load_plane = [&](int K, double (&pc)[CPT]) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) pc[c] = csrc[c] ? csrc[c][(long)K * szc] : 0.0;
    };

    // this thread's fine rows: inside the grid or not
    bool yin[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) yin[q] = j0 + rsub + q * RPP <= n && i <= n;
    // this lane's x stencil
    int xlo = 0;
    double wx[4];
    const int nx = i <= n ? stencil(i, xlo, wx) : 0;

    double W[NA][Q][4];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int q = 0; q < Q; ++q) W[a][q][0] = W[a][q][1] = W[a][q][2] = W[a][q][3] = 0.0;

    double pc[CPT];
    load_plane(Klo, pc);
    for (int K = Klo; K <= Khi; ++K) {
        // 1. plane K's coarse tile -> LDS; plane K+1's loads issued
#pragma unroll
        for (int c = 0; c < CPT; ++c)
            if (csrc[c]) C[cdst[c]] = pc[c];
        if (K < Khi) load_plane(K + 1, pc);
        // the fine planes whose stencils end at K (slot 0: 2K, slot 1:
        // 2K - 3, slot 2: plane 1 at K = 3, plane n at K = nc + 1), and
        // their u values
        int ks[3];
        bool kon[3];
        ks[0] = 2 * K;
        kon[0] = 2 * K >= 1 && 2 * K <= n;
        ks[1] = 2 * K - 3;
        kon[1] = K >= 3 && 2 * K - 3 <= n - 2;
        ks[2] = K == 3 ? 1 : n;
        kon[2] = K == 3 || K == nc + 1;
        double pu[3][NA][Q];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            kon[e] = kon[e] && ks[e] >= k0 && ks[e] < k1;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const bool on = kon[e] && yin[q];
                const long o = (long)i + (long)(j0 + rsub + q * RPP) * sy + (long)ks[e] * sz;
                pu[e][0][q] = on ? U0[o] : 0.0;
                if (NA > 1) pu[e][NA - 1][q] = on ? U1[o] : 0.0;
            }
        }
        __syncthreads();
        // 2. x pass
        for (int r = rsub; r < R; r += RPP) {
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const double *row = C + (a * RMAX + r) * CXL + xlo;
                double v = 0.0;
                if (nx == 1) v = row[0];
                else if (nx == 4) v = ((wx[0] * row[0] + wx[1] * row[1]) + wx[2] * row[2]) + wx[3] * row[3];
                X[(a * RMAX + r) * RLN + lane] = v;
            }
        }
        __syncthreads();
        // 3. y pass into the window (plane K in slot 3)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            int ylo = 0;
            double wy[4];
            const int cy = yin[q] ? stencil(j0 + rsub + q * RPP, ylo, wy) : 0;
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const double *col = X + (a * RMAX + ylo - Rlo) * RLN + lane;
                double v = 0.0;
                if (cy == 1) v = col[0];
                else if (cy == 4)
                    v = ((wy[0] * col[0] + wy[1] * col[RLN]) + wy[2] * col[2 * RLN]) + wy[3] * col[3 * RLN];
                W[a][q][0] = W[a][q][1];
                W[a][q][1] = W[a][q][2];
                W[a][q][2] = W[a][q][3];
                W[a][q][3] = v;
            }
        }
        // 4. z combinations (window slot s holds plane K - 3 + s) into u
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (!kon[e]) continue;
            const int k = ks[e];
            int lo = 0;
            double wz[4];
            const int c = stencil(k, lo, wz);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (!yin[q]) continue;
                const long o = (long)i + (long)(j0 + rsub + q * RPP) * sy + (long)k * sz;
#pragma unroll
                for (int a = 0; a < NA; ++a) {
                    const double v = c == 1 ? W[a][q][3]
                                            : ((wz[0] * W[a][q][0] + wz[1] * W[a][q][1]) + wz[2] * W[a][q][2]) +
                                                  wz[3] * W[a][q][3];
                    (a ? U1 : U0)[o] = pu[e][a][q] + v;
                }
            }
        }
    }
}

template <int NA>
hipError_t prolong4z(const Tiling &t, View<double> ec, View<double> u, View<double> ec2, View<double> u2,
                     hipStream_t s)
{
    int nmax = 0;
    long fields = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        nmax = std::max(nmax, t.seg_n(sg));
        fields += t.seg_count(sg);
    }
    if (fields == 0) return hipSuccess;
    const int rln = nmax <= 64 ? 64 : nmax <= 128 ? 128 : 256;
    // fine rows per tile, Q * BLOCK / RLN of the instantiation below (4 rows
    // measured faster than 8 at 127^3: half the registers, twice the
    // workgroups per CU)
    const int TYF = rln == 64 ? 8 : 4;
    // fine planes per chunk: about 4096 workgroups in all, at least 8 planes
    long rows = 0;
    for (int sg = 0; sg < t.nseg; ++sg) rows += (long)t.seg_count(sg) * ((t.seg_n(sg) + TYF - 1) / TYF);
    const long chunks = std::max<long>(1, std::min<long>(nmax / 8, (4096 + rows - 1) / rows));
    const int kch = (int)((nmax + chunks - 1) / chunks);
    long blocks = 0;
    for (int sg = 0; sg < t.nseg; ++sg) {
        const int n = t.seg_n(sg);
        blocks += (long)t.seg_count(sg) * ((n + TYF - 1) / TYF) * ((n + kch - 1) / kch);
    }
    const size_t lds = (size_t)NA * (TYF / 2 + 5) * ((rln / 2 + 2) + rln) * sizeof(double);
    const dim3 g((unsigned)blocks), blk(BLOCK);
    if (rln == 64) prolong4z_kernel<64, 2, NA><<<g, blk, lds, s>>>(t, kch, ec, u, ec2, u2);
    else if (rln == 128) prolong4z_kernel<128, 2, NA><<<g, blk, lds, s>>>(t, kch, ec, u, ec2, u2);
    else prolong4z_kernel<256, 4, NA><<<g, blk, lds, s>>>(t, kch, ec, u, ec2, u2);
    return hipGetLastError();
}

inline dim3 grid4(const Tiling &t) { return dim3((unsigned)grid_blocks(t)); }

#define PFMG_DISPATCH4(t, KER, ...)                                                         \
    do {                                                                                    \
        if (grid_blocks(t) == 0) return hipSuccess;                                         \
        if ((t).dim == 3) KER<3><<<grid4(t), BLOCK, 0, s>>>(__VA_ARGS__);                   \
        else KER<1><<<grid4(t), BLOCK, 0, s>>>(__VA_ARGS__);                                \
        return hipGetLastError();                                                           \
    } while (0)

}  // namespace

namespace k {

hipError_t apply_L4(const Tiling &t, double nu, View<double> u, View<double> F, hipStream_t s)
{
    PFMG_DISPATCH4(t, apply_L4_kernel, t, nu, u, F);
}

hipError_t resid4(const Tiling &t, double alpha, View<double> b, View<double> u, View<double> r, hipStream_t s)
{
    PFMG_DISPATCH4(t, resid4_kernel, t, alpha, b, u, r);
}

hipError_t smooth4(const Tiling &t, double alpha, double omega, int colour, View<double> b, View<double> src,
                   View<double> dst, hipStream_t s)
{
    if (colour > 1) return hipErrorInvalidValue;
    PFMG_DISPATCH4(t, smooth4_kernel, t, alpha, omega, colour, b, src, dst);
}

hipError_t prolong4_add(const Tiling &t, View<double> ec, View<double> u, hipStream_t s)
{
    for (int sg = 0; sg < t.nseg; ++sg)
        if (t.seg_count(sg) > 0 && (coarser(t.seg_n(sg)) < 3 || t.seg_n(sg) > 255)) return hipErrorInvalidValue;
    if (t.dim == 3) return prolong4z<1>(t, ec, u, ec, u, s);
    PFMG_DISPATCH4(t, prolong4_add_kernel, t, ec, u);
}

hipError_t prolong4_add2(const Tiling &t, View<double> ec, View<double> u, View<double> ec2, View<double> u2,
                         hipStream_t s)
{
    for (int sg = 0; sg < t.nseg; ++sg)
        if (t.seg_count(sg) > 0 && (coarser(t.seg_n(sg)) < 3 || t.seg_n(sg) > 255)) return hipErrorInvalidValue;
    if (t.dim == 3) return prolong4z<2>(t, ec, u, ec2, u2, s);
    PFMG_DISPATCH4(t, prolong4_add2_kernel, t, ec, u, ec2, u2);
}

}  // namespace k
}  // namespace pfmg
