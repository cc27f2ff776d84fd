// Network kernels of the learned initial guess (see nn.h).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: a workgroup
// of 4 wavefronts computes 64 MB output voxels (MB groups of 16 per
// wavefront) times all output channels; the K dimension runs over (tap,
// 8-channel block) groups, four per MFMA.  Each weight fragment loaded
// feeds the MB voxel groups of its wavefront, so the weights (read through
// the caches by every wavefront) cost 1/MB of their traffic per voxel.  Lane l of the MFMA holds A row l%16 and B column l%16
// with k = 8 (l/16) .. 8 (l/16) + 7, and receives D rows 4 (l/16) .. + 3 of
// column l%16.  A rows are voxels: each lane loads its voxel's 8 channels of
// one tap with one 16-byte load (channels-last); B columns are output
// channels, 16-byte loads of the weights [tap][cout][cin8].
//
// Weight gradients are GEMMs over voxels (K = voxels): 32 voxels of the
// upstream gradient and of the layer input are staged in LDS per step, so
// that the MFMA operands can be read voxel-major; one workgroup per tap and
// chunk of voxels accumulates in registers and adds its partial sums
// atomically.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nn.h"

namespace pfmg {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline long vox(int n, int s, int z, int y, int x)
{
    const long m = n + 2;
    return (((long)s * m + z) * m + y) * m + x;
}

// Domain of the M dimension of a convolution: SAME / DOWN iterate over the
// output grid; UP iterates over one parity class of the output grid.
struct Dom {
    int cz, cy, cx;
    int pz, py, px;
};

__device__ inline Dom domain(int mode, int nin, int nout, int cls)
{
    Dom d{nout, nout, nout, 0, 0, 0};
    if (mode == UP) {
        d.pz = (cls >> 2) & 1;
        d.py = (cls >> 1) & 1;
        d.px = cls & 1;
        // fine 1-based i: even i = 2 (j+1), j < nc; odd i = 2 j + 1, j <= nc
        d.cz = d.pz ? nin + 1 : nin;
        d.cy = d.py ? nin + 1 : nin;
        d.cx = d.px ? nin + 1 : nin;
    }
    return d;
}

constexpr int MB = 4;   // 16-voxel groups per wavefront

// Quotient t / d (t < 2^31) from a double reciprocal of d: the product is
// within one of the quotient, so one correction each way makes it exact.
__device__ inline unsigned udiv(unsigned t, unsigned d, double inv)
{
    unsigned q = (unsigned)((double)t * inv);
    q = q * d > t ? q - 1 : q;
    q = (q + 1) * d <= t ? q + 1 : q;
    return q;
}

// Flat index v of the M domain -> (sample, z, y, x).
struct Dec {
    unsigned cx, cy, cz;
    double ix, iy, iz;
    __device__ void operator()(unsigned v, int &s, int &z, int &y, int &x) const
    {
        const unsigned q1 = udiv(v, cx, ix), q2 = udiv(q1, cy, iy), q3 = udiv(q2, cz, iz);
        x = (int)(v - q1 * cx);
        y = (int)(q1 - q2 * cy);
        z = (int)(q2 - q3 * cz);
        s = (int)q3;
    }
};

// cb_shift: log2 of the 8-channel blocks of the input (1, 2, 4 or 8 blocks).
// Every load of a K step is issued unconditionally (a group past the end
// reads tap 0 of block 0, an A row past the end its first voxel, and the
// value is replaced by zero), and the loads of step ks + 1 are issued
// before the MFMAs of step ks.
template <int MODE, int NT>
__global__ __launch_bounds__(256) void conv_kernel(Act in, int cb_shift, Act out, const bf16 *__restrict__ W,
                                                   const float *__restrict__ bias, int relu, int batch)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nin = in.n, nout = out.n;
    constexpr int cout = NT * 16;
    const int cb_count = 1 << cb_shift;
    const Dom D = domain(MODE, nin, nout, blockIdx.y);
    const unsigned total = (unsigned)batch * (unsigned)(D.cz * D.cy * D.cx);
    const unsigned vblk = blockIdx.x * 64u * MB;
    if (vblk >= total) return;
    const Dec dec{(unsigned)D.cx, (unsigned)D.cy, (unsigned)D.cz, 1.0 / D.cx, 1.0 / D.cy, 1.0 / D.cz};
    const long m = nin + 2;
    // this lane's A row (voxel) in each of the wavefront's MB groups
    const bf16 *xin[MB];
    bool a_ok[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const unsigned va = vblk + (wave * MB + mb) * 16 + (lane & 15);
        a_ok[mb] = va < total;
        int s, iz, iy, ix;
        dec(a_ok[mb] ? va : 0u, s, iz, iy, ix);
        int bz, by, bx;   // input point (halo'd) of tap offset 0
        if (MODE == SAME) {
            bz = iz + 1; by = iy + 1; bx = ix + 1;
        } else if (MODE == DOWN) {
            bz = 2 * (iz + 1); by = 2 * (iy + 1); bx = 2 * (ix + 1);
        } else {
            // even axis: J = j + 1 (d = 0); odd axis: J = j (d = +1) or j + 1 (d = -1)
            bz = D.pz ? iz : iz + 1; by = D.py ? iy : iy + 1; bx = D.px ? ix : ix + 1;
        }
        xin[mb] = in.p + vox(nin, s, bz, by, bx) * in.cs;
    }
    const int ntap = MODE == UP ? (1 << (D.pz + D.py + D.px)) : 27;
    const int groups = ntap << cb_shift;
    const int ksteps = (groups + 3) >> 2;
    const int cin8 = cb_count * 8;
    const int kg = lane >> 4;
    // the A and B fragments of K step ks
    auto load = [&](int ks, bf16x8 (&a)[MB], bf16x8 (&bw)[NT], bool &gok) {
        const int g = ks * 4 + kg;
        gok = g < groups;
        const int gg = gok ? g : 0;
        const int t = gg >> cb_shift, cb = gg & (cb_count - 1);
        int oz, oy, ox, tapw;
        if (MODE == UP) {
            int bit = 0, wz = 0, wy = 0, wx = 0;
            oz = oy = ox = 0;
            if (D.pz) { const int sel = (t >> bit++) & 1; wz = sel ? -1 : 1; oz = sel; }
            if (D.py) { const int sel = (t >> bit++) & 1; wy = sel ? -1 : 1; oy = sel; }
            if (D.px) { const int sel = (t >> bit++) & 1; wx = sel ? -1 : 1; ox = sel; }
            tapw = (wz + 1) * 9 + (wy + 1) * 3 + (wx + 1);
        } else {
            oz = t / 9 - 1;
            oy = (t / 3) % 3 - 1;
            ox = t % 3 - 1;
            tapw = t;
        }
        const long aoff = (((long)oz * m + oy) * m + ox) * in.cs + cb * 8;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) a[mb] = *reinterpret_cast<const bf16x8 *>(xin[mb] + aoff);
#pragma unroll
        for (int q = 0; q < NT; ++q)
            bw[q] = *reinterpret_cast<const bf16x8 *>(W + ((long)tapw * cout + q * 16 + (lane & 15)) * cin8 + cb * 8);
    };
    f4 acc[MB][NT];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[mb][q] = f4{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](const bf16x8 (&a)[MB], const bf16x8 (&bw)[NT], bool gok) {
        bf16x8 az[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) az[mb] = (gok && a_ok[mb]) ? a[mb] : bf16x8{};
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int q = 0; q < NT; ++q)
                acc[mb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(az[mb], gok ? bw[q] : bf16x8{}, acc[mb][q], 0, 0, 0);
    };
    bf16x8 a0[MB], b0[NT], a1[MB], b1[NT];
    bool g0, g1;
    load(0, a0, b0, g0);
    for (int ks = 0; ks < ksteps; ks += 2) {
        // the last step's prefetch reads a group past the end (clamped)
        load(ks + 1, a1, b1, g1);
        mma(a0, b0, g0);
        if (ks + 1 >= ksteps) break;
        load(ks + 2, a0, b0, g0);
        mma(a1, b1, g1);
    }
    float bq[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) bq[q] = bias ? bias[q * 16 + (lane & 15)] : 0.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const unsigned v0 = vblk + (wave * MB + mb) * 16 + 4 * (lane >> 4);
        if (v0 >= total) continue;
        int os, oz, oy, ox;
        dec(v0, os, oz, oy, ox);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t > 0) {
                // the next voxel in the flat order
                if (++ox == D.cx) {
                    ox = 0;
                    if (++oy == D.cy) {
                        oy = 0;
                        if (++oz == D.cz) { oz = 0; ++os; }
                    }
                }
            }
            if (v0 + t >= total) break;
            int z, y, x;
            if (MODE == UP) {
                z = D.pz ? 2 * oz + 1 : 2 * (oz + 1);
                y = D.py ? 2 * oy + 1 : 2 * (oy + 1);
                x = D.px ? 2 * ox + 1 : 2 * (ox + 1);
            } else {
                z = oz + 1; y = oy + 1; x = ox + 1;
            }
            bf16 *o = out.p + vox(nout, os, z, y, x) * out.cs;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const int co = q * 16 + (lane & 15);
                float val = acc[mb][q][t] + bq[q];
                if (relu) val = fmaxf(val, 0.f);
                o[co] = (bf16)val;
            }
        }
    }
}

// SAME convolution on a tile staged in LDS: a workgroup owns a box of
// TZB x TYB x TXB output voxels of one sample (wavefront w: plane z0 + w;
// group mb: row y0 + mb; the 16 voxels of a row are the A rows).  The
// (TZB + 2) x (TYB + 2) x (TXB + 2) input voxels the box reads are loaded
// into LDS once (channels 0 .. 8 CB - 1, a voxel's channels contiguous,
// padded at 64 channels so that the 16 rows of a fragment spread over the
// banks), and every tap's A fragments are read from there; the weights
// come through the caches.  The K order is that of conv_kernel.
constexpr int TXB = 16, TYB = 4, TZB = 4;
constexpr int BXB = TXB + 2, BYB = TYB + 2, BZB = TZB + 2;

__host__ __device__ constexpr int tile_vstride(int cb) { return 8 * cb + (cb >= 8 ? 8 : 0); }

template <int NT, int CB>
__global__ __launch_bounds__(256) void conv_same_lds_kernel(Act in, Act out, const bf16 *__restrict__ W,
                                                            const float *__restrict__ bias, int relu)
{
    static_assert(MB == TYB && TZB == 4, "one plane per wavefront, one row per group");
    constexpr int C8 = 8 * CB, VS = tile_vstride(CB);
    constexpr int cout = NT * 16;
    extern __shared__ unsigned char smem_raw[];
    bf16 *tile = reinterpret_cast<bf16 *>(smem_raw);   // [BZB][BYB][BXB] voxels of VS channels
    const int n = in.n;
    const int nbx = (n + TXB - 1) / TXB, nby = (n + TYB - 1) / TYB, nbz = (n + TZB - 1) / TZB;
    unsigned b = blockIdx.x;
    const int bx = (int)(b % (unsigned)nbx);
    b /= (unsigned)nbx;
    const int by = (int)(b % (unsigned)nby);
    b /= (unsigned)nby;
    const int bz = (int)(b % (unsigned)nbz);
    const int s = (int)(b / (unsigned)nbz);
    const int x0 = bx * TXB, y0 = by * TYB, z0 = bz * TZB;   // first output voxel (0-based interior)

    // stage the box: halo'd input voxel (z0 + vz, y0 + vy, x0 + vx), clamped
    // to the tensor (clamped voxels only feed outputs past the grid)
    constexpr int CHUNKS = BZB * BYB * BXB * CB;
    constexpr int PER = (CHUNKS + 255) / 256;
    constexpr int BATCH = PER < 8 ? PER : 8;
    for (int p0 = 0; p0 < PER; p0 += BATCH) {
        bf16x8 v[BATCH];
        int dst[BATCH];
#pragma unroll
        for (int e = 0; e < BATCH; ++e) {
            const int c = (int)threadIdx.x + (p0 + e) * 256;
            const int cc = c < CHUNKS ? c : CHUNKS - 1;
            const int cb = cc % CB, vv = cc / CB;
            const int vx = vv % BXB, vy = (vv / BXB) % BYB, vz = vv / (BXB * BYB);
            const int gz = min(z0 + vz, n + 1), gy = min(y0 + vy, n + 1), gx = min(x0 + vx, n + 1);
            v[e] = *reinterpret_cast<const bf16x8 *>(in.p + vox(n, s, gz, gy, gx) * in.cs + cb * 8);
            dst[e] = c < CHUNKS && p0 + e < PER ? vv * VS + cb * 8 : -1;
        }
#pragma unroll
        for (int e = 0; e < BATCH; ++e)
            if (dst[e] >= 0) *reinterpret_cast<bf16x8 *>(tile + dst[e]) = v[e];
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kg = lane >> 4, v = lane & 15;
    constexpr int groups = 27 * CB, ksteps = (groups + 3) / 4;
    f4 acc[MB][NT];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[mb][q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < ksteps; ++ks) {
        const int g = ks * 4 + kg;
        const bool gok = g < groups;
        const int gg = gok ? g : 0;
        const int t = gg / CB, cb = gg % CB;
        const int oz = t / 9, oy = (t / 3) % 3, ox = t % 3;   // box offsets 0..2 (tap offset + 1)
        bf16x8 a[MB], bw[NT];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int vv = ((wave + oz) * BYB + (mb + oy)) * BXB + (v + ox);
            a[mb] = *reinterpret_cast<const bf16x8 *>(tile + vv * VS + cb * 8);
        }
#pragma unroll
        for (int q = 0; q < NT; ++q)
            bw[q] = *reinterpret_cast<const bf16x8 *>(W + ((long)t * cout + q * 16 + v) * C8 + cb * 8);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int q = 0; q < NT; ++q)
                acc[mb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gok ? a[mb] : bf16x8{}, gok ? bw[q] : bf16x8{},
                                                                     acc[mb][q], 0, 0, 0);
    }
    float bq[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) bq[q] = bias ? bias[q * 16 + v] : 0.f;
    const int z = z0 + wave;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int y = y0 + mb;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int x = x0 + 4 * kg + t;
            if (x >= n || y >= n || z >= n) continue;
            bf16 *o = out.p + vox(n, s, z + 1, y + 1, x + 1) * out.cs;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                float val = acc[mb][q][t] + bq[q];
                if (relu) val = fmaxf(val, 0.f);
                o[q * 16 + v] = (bf16)val;
            }
        }
    }
}

// UP convolution (coarse -> fine) on a coarse box staged in LDS: a
// workgroup of 8 wavefronts owns a fine box of 4 x 4 x 32 points starting
// at fine (4 bz + 1, 4 by + 1, 32 bx + 1); wavefront w takes the parity
// class (pz, py, px) = bits of w, i.e. 2 x 2 of the box's rows and 16 of
// the 32 points of each (every other x), so the four groups of a
// wavefront share their taps.  Per axis, fine 2J + 1 reads coarse J
// (d = +1) and J + 1 (d = -1), fine 2J reads J (d = 0); the box reads
// coarse 2 bz .. 2 bz + 2, 2 by .. 2 by + 2, 16 bx .. 16 bx + 16.
constexpr int UXB = 32, UCX = UXB / 2 + 1;

template <int NT, int CB>
__global__ __launch_bounds__(512) void conv_up_lds_kernel(Act in, Act out, const bf16 *__restrict__ W,
                                                          const float *__restrict__ bias, int relu)
{
    constexpr int C8 = 8 * CB, VS = tile_vstride(CB);
    constexpr int cout = NT * 16;
    constexpr int cb_shift = CB == 1 ? 0 : CB == 2 ? 1 : CB == 4 ? 2 : 3;
    extern __shared__ unsigned char smem_raw[];
    bf16 *tile = reinterpret_cast<bf16 *>(smem_raw);   // [3][3][UCX] coarse voxels of VS channels
    const int nc = in.n, nf = out.n;
    const int nbx = (nf + UXB - 1) / UXB, nby = (nf + 3) / 4, nbz = (nf + 3) / 4;
    unsigned b = blockIdx.x;
    const int bx = (int)(b % (unsigned)nbx);
    b /= (unsigned)nbx;
    const int by = (int)(b % (unsigned)nby);
    b /= (unsigned)nby;
    const int bz = (int)(b % (unsigned)nbz);
    const int s = (int)(b / (unsigned)nbz);
    const int cz0 = 2 * bz, cy0 = 2 * by, cx0 = 16 * bx;   // first coarse (halo'd) index of the box

    constexpr int CHUNKS = 3 * 3 * UCX * CB;
    for (int c = threadIdx.x; c < CHUNKS; c += 512) {
        const int cb = c % CB, vv = c / CB;
        const int vx = vv % UCX, vy = (vv / UCX) % 3, vz = vv / (UCX * 3);
        const int gz = min(cz0 + vz, nc + 1), gy = min(cy0 + vy, nc + 1), gx = min(cx0 + vx, nc + 1);
        *reinterpret_cast<bf16x8 *>(tile + vv * VS + cb * 8) =
            *reinterpret_cast<const bf16x8 *>(in.p + vox(nc, s, gz, gy, gx) * in.cs + cb * 8);
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kg = lane >> 4, v = lane & 15;
    const int pz = (wave >> 2) & 1, py = (wave >> 1) & 1, px = wave & 1;
    const int ntap = 1 << (pz + py + px);
    const int groups = ntap << cb_shift;
    const int ksteps = (groups + 3) >> 2;
    // group mb = (zr, yr): fine row 2 c + 1 + 2 r + (1 - p) on each axis,
    // whose base coarse index in the box is r (odd) or 1 + r (even)
    f4 acc[MB][NT];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[mb][q] = f4{0.f, 0.f, 0.f, 0.f};
    const int xb = px ? v : v + 1;
    for (int ks = 0; ks < ksteps; ++ks) {
        const int g = ks * 4 + kg;
        const bool gok = g < groups;
        const int gg = gok ? g : 0;
        const int t = gg >> cb_shift, cb = gg & (CB - 1);
        int bit = 0, oz = 0, oy = 0, ox = 0, wz = 1, wy = 1, wx = 1;   // offsets; weight index per axis
        if (pz) { const int sel = (t >> bit++) & 1; oz = sel; wz = sel ? 0 : 2; }
        if (py) { const int sel = (t >> bit++) & 1; oy = sel; wy = sel ? 0 : 2; }
        if (px) { const int sel = (t >> bit++) & 1; ox = sel; wx = sel ? 0 : 2; }
        const int tapw = wz * 9 + wy * 3 + wx;
        bf16x8 a[MB], bw[NT];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int zr = mb >> 1, yr = mb & 1;
            const int zb = pz ? zr : 1 + zr, yb = py ? yr : 1 + yr;
            const int vv = ((zb + oz) * 3 + (yb + oy)) * UCX + (xb + ox);
            a[mb] = *reinterpret_cast<const bf16x8 *>(tile + vv * VS + cb * 8);
        }
#pragma unroll
        for (int q = 0; q < NT; ++q)
            bw[q] = *reinterpret_cast<const bf16x8 *>(W + ((long)tapw * cout + q * 16 + v) * C8 + cb * 8);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int q = 0; q < NT; ++q)
                acc[mb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gok ? a[mb] : bf16x8{}, gok ? bw[q] : bf16x8{},
                                                                     acc[mb][q], 0, 0, 0);
    }
    float bq[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) bq[q] = bias ? bias[q * 16 + v] : 0.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int zr = mb >> 1, yr = mb & 1;
        const int z = 4 * bz + 1 + 2 * zr + (1 - pz), y = 4 * by + 1 + 2 * yr + (1 - py);   // fine, 1-based
        if (z > nf || y > nf) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int x = UXB * bx + 1 + 2 * (4 * kg + t) + (1 - px);
            if (x > nf) continue;
            bf16 *o = out.p + vox(nf, s, z, y, x) * out.cs;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                float val = acc[mb][q][t] + bq[q];
                if (relu) val = fmaxf(val, 0.f);
                o[q * 16 + v] = (bf16)val;
            }
        }
    }
}

// Weight gradient of one tap over a chunk of the base domain: SAME and DOWN
// iterate over the output grid (dz at the point, x at the tap's input
// point); UP iterates over the coarse input grid (x at J, dz at 2J + d).
constexpr int WG_K = 32;
constexpr int WG_LD = 64 + 8;   // LDS row length (bf16), padded

template <int MODE>
__global__ __launch_bounds__(256) void wgrad_kernel(Act x, int cin, Act dz, int cout, float *__restrict__ dW,
                                                    int batch, long chunk)
{
    __shared__ bf16 sz[WG_K][WG_LD];
    __shared__ bf16 sx[WG_K][WG_LD];
    const int tap = blockIdx.y;
    const int tz = tap / 9 - 1, ty = (tap / 3) % 3 - 1, tx = tap % 3 - 1;
    const int nb = MODE == UP ? x.n : dz.n;
    const long total = (long)batch * nb * nb * nb;
    const long vb = (long)blockIdx.x * chunk;
    if (vb >= total) return;
    const long ve = vb + chunk < total ? vb + chunk : total;
    const int cin16 = (cin + 15) & ~15;
    const int cin8 = (cin + 7) & ~7;
    const int MT = cout / 16, NTI = cin16 / 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    f4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    const int zv = cout / 8, xv = cin16 / 8;
    for (long v = vb; v < ve; v += WG_K) {
        for (int idx = threadIdx.x; idx < WG_K * (zv + xv); idx += 256) {
            const bool isz = idx < WG_K * zv;
            const int j = isz ? idx : idx - WG_K * zv;
            const int per = isz ? zv : xv;
            const int k = j / per, c8 = j - k * per;
            const long vv = v + k;
            bf16x8 val = {};
            if (vv < ve && (isz || c8 * 8 < cin8)) {
                long t = vv;
                const int ox = (int)(t % nb);
                t /= nb;
                const int oy = (int)(t % nb);
                t /= nb;
                const int oz = (int)(t % nb);
                const int s = (int)(t / nb);
                int pz, py, px;
                const Act &A = isz ? dz : x;
                if (isz) {
                    if (MODE == UP) { pz = 2 * (oz + 1) + tz; py = 2 * (oy + 1) + ty; px = 2 * (ox + 1) + tx; }
                    else { pz = oz + 1; py = oy + 1; px = ox + 1; }
                } else {
                    if (MODE == SAME) { pz = oz + 1 + tz; py = oy + 1 + ty; px = ox + 1 + tx; }
                    else if (MODE == DOWN) { pz = 2 * (oz + 1) + tz; py = 2 * (oy + 1) + ty; px = 2 * (ox + 1) + tx; }
                    else { pz = oz + 1; py = oy + 1; px = ox + 1; }
                }
                val = *reinterpret_cast<const bf16x8 *>(A.p + vox(A.n, s, pz, py, px) * A.cs + c8 * 8);
            }
            bf16 *dst = isz ? &sz[k][c8 * 8] : &sx[k][c8 * 8];
#pragma unroll
            for (int e = 0; e < 8; ++e) dst[e] = val[e];
        }
        __syncthreads();
        int slot = 0;
        for (int tile = wave; tile < MT * NTI; tile += 4, ++slot) {
            const int mt = tile / NTI, nt = tile - mt * NTI;
            bf16x8 a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = sz[(lane >> 4) * 8 + e][mt * 16 + (lane & 15)];
                b[e] = sx[(lane >> 4) * 8 + e][nt * 16 + (lane & 15)];
            }
            if (slot == 0) acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[0], 0, 0, 0);
            else if (slot == 1) acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[1], 0, 0, 0);
            else if (slot == 2) acc[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[2], 0, 0, 0);
            else acc[3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[3], 0, 0, 0);
        }
        __syncthreads();
    }
    int slot = 0;
    for (int tile = wave; tile < MT * NTI; tile += 4, ++slot) {
        const int mt = tile / NTI, nt = tile - mt * NTI;
        const int ci = nt * 16 + (lane & 15);
        if (ci >= cin) continue;
        const f4 r = slot == 0 ? acc[0] : slot == 1 ? acc[1] : slot == 2 ? acc[2] : acc[3];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int co = mt * 16 + 4 * (lane >> 4) + t;
            atomicAdd(dW + ((long)tap * cout + co) * cin + ci, r[t]);
        }
    }
}

__global__ void bias_grad_kernel(Act dz, int cout, float *db, long total, long chunk)
{
    __shared__ float part[256];
    const int c = threadIdx.x % cout, lanes = 256 / cout, sub = threadIdx.x / cout;
    const long vb = (long)blockIdx.x * chunk;
    const long ve = vb + chunk < total ? vb + chunk : total;
    const int n = dz.n;
    float acc = 0.f;
    if (sub < lanes)
        for (long v = vb + sub; v < ve; v += lanes) {
            long t = v;
            const int ox = (int)(t % n);
            t /= n;
            const int oy = (int)(t % n);
            t /= n;
            const int oz = (int)(t % n);
            const int s = (int)(t / n);
            acc += (float)dz.p[vox(n, s, oz + 1, oy + 1, ox + 1) * dz.cs + c];
        }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < cout) {
        float sum = 0.f;
        for (int q = 0; q < lanes; ++q) sum += part[q * cout + threadIdx.x];
        atomicAdd(db + threadIdx.x, sum);
    }
}

__global__ void relu_bwd_kernel(Act dy, Act dsk, Act y, Act dz, int c, long total)
{
    const long w = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int groups = c / 8;
    if (w >= total * groups) return;
    const int g = (int)(w % groups);
    long t = w / groups;
    const int n = y.n;
    const int ox = (int)(t % n);
    t /= n;
    const int oy = (int)(t % n);
    t /= n;
    const int oz = (int)(t % n);
    const int s = (int)(t / n);
    const long vv = vox(n, s, oz + 1, oy + 1, ox + 1);
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(dy.p + vv * dy.cs + g * 8);
    const bf16x8 yy = *reinterpret_cast<const bf16x8 *>(y.p + vv * y.cs + g * 8);
    bf16x8 k = {};
    if (dsk.p) k = *reinterpret_cast<const bf16x8 *>(dsk.p + vv * dsk.cs + g * 8);
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float v = (float)a[e] + (dsk.p ? (float)k[e] : 0.f);
        r[e] = (bf16)((float)yy[e] > 0.f ? v : 0.f);
    }
    *reinterpret_cast<bf16x8 *>(dz.p + vv * dz.cs + g * 8) = r;
}

__global__ void pw_forward_kernel(Act x, const float *__restrict__ w, const float *__restrict__ b, float *y, long total)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= total) return;
    const int n = x.n;
    long t = v;
    const int ox = (int)(t % n);
    t /= n;
    const int oy = (int)(t % n);
    t /= n;
    const int oz = (int)(t % n);
    const int s = (int)(t / n);
    const bf16 *p = x.p + vox(n, s, oz + 1, oy + 1, ox + 1) * x.cs;
    const bf16x8 lo = *reinterpret_cast<const bf16x8 *>(p), hi = *reinterpret_cast<const bf16x8 *>(p + 8);
    float acc = b[0];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc += w[e] * (float)lo[e] + w[8 + e] * (float)hi[e];
    y[v] = acc;
}

__global__ void pw_loss_backward_kernel(Act x, const float *__restrict__ w, const float *__restrict__ y,
                                        const float *__restrict__ tg, float scale, Act dx, float *dw, float *db,
                                        double *loss, long total)
{
    __shared__ float part[18][256];
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float contrib[16] = {}, g = 0.f, l2 = 0.f;
    if (v < total) {
        const int n = x.n;
        long t = v;
        const int ox = (int)(t % n);
        t /= n;
        const int oy = (int)(t % n);
        t /= n;
        const int oz = (int)(t % n);
        const int s = (int)(t / n);
        const long vv = vox(n, s, oz + 1, oy + 1, ox + 1);
        const float r = y[v] - tg[v];
        l2 = r * r;
        g = scale * r;
        const bf16 *p = x.p + vv * x.cs;
        const bf16x8 lo = *reinterpret_cast<const bf16x8 *>(p), hi = *reinterpret_cast<const bf16x8 *>(p + 8);
        bf16x8 dlo, dhi;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            contrib[e] = g * (float)lo[e];
            contrib[8 + e] = g * (float)hi[e];
            dlo[e] = (bf16)(g * w[e]);
            dhi[e] = (bf16)(g * w[8 + e]);
        }
        bf16 *q = dx.p + vv * dx.cs;
        *reinterpret_cast<bf16x8 *>(q) = dlo;
        *reinterpret_cast<bf16x8 *>(q + 8) = dhi;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) part[e][threadIdx.x] = contrib[e];
    part[16][threadIdx.x] = g;
    part[17][threadIdx.x] = l2;
    __syncthreads();
    if (threadIdx.x < 18) {
        float sum = 0.f;
        for (int q = 0; q < (int)blockDim.x; ++q) sum += part[threadIdx.x][q];
        if (threadIdx.x < 16) atomicAdd(dw + threadIdx.x, sum);
        else if (threadIdx.x == 16) atomicAdd(db, sum);
        else atomicAdd(loss, (double)sum);
    }
}

__global__ void weights_forward_kernel(const float *Wm, int cout, int cin, int cin8, bf16 *Wf)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = 27L * cout * cin8;
    if (i >= total) return;
    const int ci = (int)(i % cin8);
    const long r = i / cin8;   // tap * cout + co
    Wf[i] = (bf16)(ci < cin ? Wm[r * cin + ci] : 0.f);
}

__global__ void weights_backward_kernel(const float *Wm, int cout, int cin, int flip, bf16 *Wb)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = 27L * cout * cin;
    if (i >= total) return;
    // destination [tap'][ci][co]
    const int co = (int)(i % cout);
    const long r = i / cout;
    const int ci = (int)(r % cin);
    const int tp = (int)(r / cin);
    const int tap = flip ? 26 - tp : tp;
    Wb[i] = (bf16)Wm[((long)tap * cout + co) * cin + ci];
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, long count, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void fill_f32_kernel(float *p, float v, long count)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---- field <-> network (3D fields in the solver layout)
__global__ __launch_bounds__(BLOCK) void make_input_kernel(Tiling t, double alpha, View<double> b, View<double> u,
                                                           const double *sr, const double *su, Act x0)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<3>(t, q, i, j, k, o)) return;
    const double *uu = fp(u, q);
    const double ah = q.par(alpha) * (double)(q.n + 1) * (double)(q.n + 1);
    const double hu = uu[o] - ah * d2sum<3>(uu, o, row_stride(q.n), plane_stride(q.n));
    const double r = fp(b, q)[o] - hu;
    bf16x8 v = {};
    v[0] = (bf16)(float)(r / sr[q.item]);
    v[1] = (bf16)(float)(uu[o] / su[q.item]);
    v[2] = (bf16)(float)ah;
    *reinterpret_cast<bf16x8 *>(x0.p + vox(q.n, q.item, k, j, i) * x0.cs) = v;
}

__global__ __launch_bounds__(BLOCK) void apply_guess_kernel(Tiling t, View<double> u, const float *y,
                                                            const double *sr, View<double> g)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<3>(t, q, i, j, k, o)) return;
    const long n = q.n;
    const long d = (i - 1) + n * ((j - 1) + n * (long)(k - 1));
    fp(g, q)[o] = fp(u, q)[o] + sr[q.item] * (double)y[(long)q.item * n * n * n + d];
}

__global__ void gather_batch_kernel(const bf16 *pairs, const float *ah2, const int *idx, int n, Act x0, float *tg,
                                    long total)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= total) return;
    const long n3 = (long)n * n * n;
    const int s = (int)(v / n3);
    const long d = v - s * n3;
    const int ox = (int)(d % n), oy = (int)((d / n) % n), oz = (int)(d / ((long)n * n));
    const long pr = idx[s];
    bf16x8 val = {};
    val[0] = pairs[(pr * 3 + 0) * n3 + d];
    val[1] = pairs[(pr * 3 + 1) * n3 + d];
    val[2] = (bf16)ah2[pr];
    *reinterpret_cast<bf16x8 *>(x0.p + vox(n, s, oz + 1, oy + 1, ox + 1) * x0.cs) = val;
    tg[v] = (float)pairs[(pr * 3 + 2) * n3 + d];
}

__global__ void act_to_dense_kernel(Act a, int c, float *dst, long total)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= total) return;
    const int n = a.n;
    const long n3 = (long)n * n * n;
    const int s = (int)(v / n3);
    const long d = v - s * n3;
    const int ox = (int)(d % n), oy = (int)((d / n) % n), oz = (int)(d / ((long)n * n));
    const bf16 *p = a.p + vox(n, s, oz + 1, oy + 1, ox + 1) * a.cs;
    for (int q = 0; q < c; ++q) dst[((long)s * c + q) * n3 + d] = (float)p[q];
}

__global__ void load_input_dense_kernel(const float *xd, int n, Act x0, long total)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= total) return;
    const long n3 = (long)n * n * n;
    const int s = (int)(v / n3);
    const long d = v - s * n3;
    const int ox = (int)(d % n), oy = (int)((d / n) % n), oz = (int)(d / ((long)n * n));
    bf16x8 val = {};
#pragma unroll
    for (int c = 0; c < 3; ++c) val[c] = (bf16)xd[((long)s * 3 + c) * n3 + d];
    *reinterpret_cast<bf16x8 *>(x0.p + vox(n, s, oz + 1, oy + 1, ox + 1) * x0.cs) = val;
}

__global__ __launch_bounds__(BLOCK) void record_inputs_kernel(Tiling t, double alpha, View<double> b, View<double> u,
                                                              const double *sr, const double *su, bf16 *pairs,
                                                              float *ah2, long slot0, double *u0)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<3>(t, q, i, j, k, o)) return;
    const long n = q.n, n3 = n * n * n;
    const long d = (i - 1) + n * ((j - 1) + n * (long)(k - 1));
    const double *uu = fp(u, q);
    const double ah = q.par(alpha) * (double)(n + 1) * (double)(n + 1);
    const double r = fp(b, q)[o] - (uu[o] - ah * d2sum<3>(uu, o, row_stride(q.n), plane_stride(q.n)));
    const long slot = slot0 + q.item;
    pairs[(slot * 3 + 0) * n3 + d] = (bf16)(float)(r / sr[q.item]);
    pairs[(slot * 3 + 1) * n3 + d] = (bf16)(float)(uu[o] / su[q.item]);
    u0[(long)q.item * n3 + d] = uu[o];
    if (d == 0) ah2[slot] = (float)ah;
}

__global__ __launch_bounds__(BLOCK) void record_target_kernel(Tiling t, View<double> u, const double *sr,
                                                              const double *u0, bf16 *pairs, long slot0)
{
    Pt q; int i, j, k; long o;
    if (!tile_point<3>(t, q, i, j, k, o)) return;
    const long n = q.n, n3 = n * n * n;
    const long d = (i - 1) + n * ((j - 1) + n * (long)(k - 1));
    const long slot = slot0 + q.item;
    pairs[(slot * 3 + 2) * n3 + d] = (bf16)(float)((fp(u, q)[o] - u0[(long)q.item * n3 + d]) / sr[q.item]);
}

inline unsigned blocks_of(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t conv(Mode mode, const Act &in, int cin8, const Act &out, int cout, const bf16 *W, const float *bias,
                bool relu, int batch, hipStream_t s)
{
    if (cin8 % 8 || cout % 16 || cout > 64 || in.cs % 8 || out.cs % 8 || batch < 1) return hipErrorInvalidValue;
    if (mode == SAME && in.n != out.n) return hipErrorInvalidValue;
    if (mode == DOWN && out.n != (in.n + 1) / 2 - 1) return hipErrorInvalidValue;
    if (mode == UP && in.n != (out.n + 1) / 2 - 1) return hipErrorInvalidValue;
    const int cb = cin8 / 8;
    if (cb & (cb - 1)) return hipErrorInvalidValue;   // 1, 2, 4 or 8 channel blocks
    const int cb_shift = __builtin_ctz((unsigned)cb);
    long total;
    dim3 grid;
    if (mode == UP) {
        total = (long)batch * (in.n + 1) * (in.n + 1) * (in.n + 1);
        grid = dim3(blocks_of(total, 64 * MB), 8);
    } else {
        total = (long)batch * out.n * out.n * out.n;
        grid = dim3(blocks_of(total, 64 * MB), 1);
    }
    const int r = relu ? 1 : 0;
    if (mode == SAME) {
        // LDS-tiled kernel: (n/4)^2 (n/16) boxes per sample
        const int nb = ((out.n + TXB - 1) / TXB) * ((out.n + TYB - 1) / TYB) * ((out.n + TZB - 1) / TZB);
        const dim3 g2((unsigned)((long)nb * batch));
        const size_t lds = (size_t)BZB * BYB * BXB * tile_vstride(cb) * sizeof(bf16);
#define NN_SAME(NT_, CB_)                                                                                    \
    do {                                                                                                     \
        static const hipError_t ea = hipFuncSetAttribute((const void *)conv_same_lds_kernel<NT_, CB_>,      \
                                                          hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024); \
        if (ea != hipSuccess) return ea;                                                                     \
        conv_same_lds_kernel<NT_, CB_><<<g2, 256, lds, s>>>(in, out, W, bias, r);                            \
    } while (0)
#define NN_SAME_CB(NT_)                          \
    switch (cb) {                                \
    case 1: NN_SAME(NT_, 1); break;              \
    case 2: NN_SAME(NT_, 2); break;              \
    case 4: NN_SAME(NT_, 4); break;              \
    default: NN_SAME(NT_, 8); break;             \
    }
        switch (cout / 16) {
        case 1: NN_SAME_CB(1); break;
        case 2: NN_SAME_CB(2); break;
        case 3: NN_SAME_CB(3); break;
        default: NN_SAME_CB(4); break;
        }
#undef NN_SAME_CB
#undef NN_SAME
        return hipGetLastError();
    }
    if (mode == UP) {
        // coarse-box kernel: fine boxes of 4 x 4 x 32 points
        const int nf = out.n;
        const long nb = (long)((nf + UXB - 1) / UXB) * ((nf + 3) / 4) * ((nf + 3) / 4);
        const dim3 g2((unsigned)(nb * batch));
        const size_t lds = (size_t)3 * 3 * UCX * tile_vstride(cb) * sizeof(bf16);
#define NN_UP(NT_, CB_) conv_up_lds_kernel<NT_, CB_><<<g2, 512, lds, s>>>(in, out, W, bias, r)
#define NN_UP_CB(NT_)                            \
    switch (cb) {                                \
    case 1: NN_UP(NT_, 1); break;                \
    case 2: NN_UP(NT_, 2); break;                \
    case 4: NN_UP(NT_, 4); break;                \
    default: NN_UP(NT_, 8); break;               \
    }
        switch (cout / 16) {
        case 1: NN_UP_CB(1); break;
        case 2: NN_UP_CB(2); break;
        case 3: NN_UP_CB(3); break;
        default: NN_UP_CB(4); break;
        }
#undef NN_UP_CB
#undef NN_UP
        return hipGetLastError();
    }
#define NN_CONV(MODE_, NT_) conv_kernel<MODE_, NT_><<<grid, 256, 0, s>>>(in, cb_shift, out, W, bias, r, batch)
#define NN_CONV_NT(MODE_)                     \
    switch (cout / 16) {                      \
    case 1: NN_CONV(MODE_, 1); break;         \
    case 2: NN_CONV(MODE_, 2); break;         \
    case 3: NN_CONV(MODE_, 3); break;         \
    default: NN_CONV(MODE_, 4); break;        \
    }
    if (mode == SAME) NN_CONV_NT(SAME)
    else if (mode == DOWN) NN_CONV_NT(DOWN)
    else NN_CONV_NT(UP)
#undef NN_CONV_NT
#undef NN_CONV
    return hipGetLastError();
}

hipError_t conv_wgrad(Mode mode, const Act &x, int cin, const Act &dz, int cout, float *dW, int batch, hipStream_t s)
{
    if (cout % 16 || cout > 64 || cin > 64 || cin < 1 || x.cs % 8 || dz.cs % 8) return hipErrorInvalidValue;
    if ((cout / 16) * ((cin + 15) / 16) > 16) return hipErrorInvalidValue;
    const int nb = mode == UP ? x.n : dz.n;
    const long total = (long)batch * nb * nb * nb;
    const long chunk = std::max<long>(WG_K, ((total + 255) / 256 + WG_K - 1) / WG_K * WG_K);
    const dim3 grid(blocks_of(total, (int)chunk), 27);
    if (mode == SAME) wgrad_kernel<SAME><<<grid, 256, 0, s>>>(x, cin, dz, cout, dW, batch, chunk);
    else if (mode == DOWN) wgrad_kernel<DOWN><<<grid, 256, 0, s>>>(x, cin, dz, cout, dW, batch, chunk);
    else wgrad_kernel<UP><<<grid, 256, 0, s>>>(x, cin, dz, cout, dW, batch, chunk);
    return hipGetLastError();
}

hipError_t bias_grad(const Act &dz, int cout, float *db, int batch, hipStream_t s)
{
    if (cout < 1 || cout > 256 || 256 % cout) return hipErrorInvalidValue;
    const long total = (long)batch * dz.n * dz.n * dz.n;
    const long chunk = std::max<long>(256, (total + 511) / 512);
    bias_grad_kernel<<<blocks_of(total, (int)chunk), 256, 0, s>>>(dz, cout, db, total, chunk);
    return hipGetLastError();
}

hipError_t relu_bwd(const Act &dy, const Act &dskip, const Act &y, const Act &dz, int c, int batch, hipStream_t s)
{
    if (c % 8) return hipErrorInvalidValue;
    const long total = (long)batch * y.n * y.n * y.n;
    relu_bwd_kernel<<<blocks_of(total * (c / 8), 256), 256, 0, s>>>(dy, dskip, y, dz, c, total);
    return hipGetLastError();
}

hipError_t pw_forward(const Act &x, const float *w, const float *b, float *y, int batch, hipStream_t s)
{
    const long total = (long)batch * x.n * x.n * x.n;
    pw_forward_kernel<<<blocks_of(total, 256), 256, 0, s>>>(x, w, b, y, total);
    return hipGetLastError();
}

hipError_t pw_loss_backward(const Act &x, const float *w, const float *y, const float *t, double count, const Act &dx,
                            float *dw, float *db, double *loss_acc, int batch, hipStream_t s)
{
    const long total = (long)batch * x.n * x.n * x.n;
    pw_loss_backward_kernel<<<blocks_of(total, 256), 256, 0, s>>>(x, w, y, t, (float)(2.0 / count), dx, dw, db,
                                                                   loss_acc, total);
    return hipGetLastError();
}

hipError_t weights_forward(const float *Wm, int cout, int cin, int cin8, bf16 *Wf, hipStream_t s)
{
    weights_forward_kernel<<<blocks_of(27L * cout * cin8, 256), 256, 0, s>>>(Wm, cout, cin, cin8, Wf);
    return hipGetLastError();
}

hipError_t weights_backward(const float *Wm, int cout, int cin, bool flip, bf16 *Wb, hipStream_t s)
{
    weights_backward_kernel<<<blocks_of(27L * cout * cin, 256), 256, 0, s>>>(Wm, cout, cin, flip ? 1 : 0, Wb);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m, float *v, long count, float lr, float beta1, float beta2,
                float eps, int t, hipStream_t s)
{
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    adam_kernel<<<blocks_of(count, 256), 256, 0, s>>>(p, g, m, v, count, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t fill_f32(float *p, float v, long count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    fill_f32_kernel<<<blocks_of(count, 256), 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}

hipError_t make_input(const Tiling &t, double alpha, View<double> b, View<double> u, const double *sr,
                      const double *su, const Act &x0, hipStream_t s)
{
    if (t.dim != 3 || t.nseg != 1 || x0.n != t.n || x0.cs < 8) return hipErrorInvalidValue;
    const long nb = grid_blocks(t);
    if (nb == 0) return hipSuccess;
    make_input_kernel<<<(unsigned)nb, BLOCK, 0, s>>>(t, alpha, b, u, sr, su, x0);
    return hipGetLastError();
}

hipError_t apply_guess(const Tiling &t, View<double> u, const float *y, const double *sr, View<double> g,
                       hipStream_t s)
{
    if (t.dim != 3 || t.nseg != 1) return hipErrorInvalidValue;
    const long nb = grid_blocks(t);
    if (nb == 0) return hipSuccess;
    apply_guess_kernel<<<(unsigned)nb, BLOCK, 0, s>>>(t, u, y, sr, g);
    return hipGetLastError();
}

hipError_t gather_batch(const bf16 *pairs, const float *ah2, const int *idx, int batch, int n, const Act &x0,
                        float *target, hipStream_t s)
{
    if (x0.n != n || x0.cs < 8) return hipErrorInvalidValue;
    const long total = (long)batch * n * n * n;
    gather_batch_kernel<<<blocks_of(total, 256), 256, 0, s>>>(pairs, ah2, idx, n, x0, target, total);
    return hipGetLastError();
}

hipError_t act_to_dense(const Act &a, int c, int batch, float *dst, hipStream_t s)
{
    const long total = (long)batch * a.n * a.n * a.n;
    act_to_dense_kernel<<<blocks_of(total, 256), 256, 0, s>>>(a, c, dst, total);
    return hipGetLastError();
}

hipError_t load_input_dense(const float *xd, int batch, int n, const Act &x0, hipStream_t s)
{
    if (x0.n != n || x0.cs < 8) return hipErrorInvalidValue;
    const long total = (long)batch * n * n * n;
    load_input_dense_kernel<<<blocks_of(total, 256), 256, 0, s>>>(xd, n, x0, total);
    return hipGetLastError();
}

hipError_t record_inputs(const Tiling &t, double alpha, View<double> b, View<double> u, const double *sr,
                         const double *su, bf16 *pairs, float *ah2, long slot0, double *u0, hipStream_t s)
{
    if (t.dim != 3 || t.nseg != 1) return hipErrorInvalidValue;
    const long nb = grid_blocks(t);
    if (nb == 0) return hipSuccess;
    record_inputs_kernel<<<(unsigned)nb, BLOCK, 0, s>>>(t, alpha, b, u, sr, su, pairs, ah2, slot0, u0);
    return hipGetLastError();
}

hipError_t record_target(const Tiling &t, View<double> u, const double *sr, const double *u0, bf16 *pairs, long slot0,
                         hipStream_t s)
{
    if (t.dim != 3 || t.nseg != 1) return hipErrorInvalidValue;
    const long nb = grid_blocks(t);
    if (nb == 0) return hipSuccess;
    record_target_kernel<<<(unsigned)nb, BLOCK, 0, s>>>(t, u, sr, u0, pairs, slot0);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace pfmg
