// Point-per-thread tiling shared by the grid kernels.
//
// A launch covers `count` fields of one grid.  3D: a workgroup of 256
// threads (4 wavefronts) owns a 64 x 4 patch of one z-plane of one field,
// one wavefront per 64-point row segment, so every wavefront reads and
// writes whole 512-byte (FP64) row segments.  1D: 256 consecutive points.
//
// The flat workgroup id is remapped so that each of the 8 XCDs (which
// receive workgroups round-robin) gets one contiguous run of tiles: the
// planes k-1, k, k+1 of a tile and the neighbouring rows then mostly meet
// in the same XCD's L2.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.h"

namespace pfmg {

constexpr int TILE_X = 64;
constexpr int TILE_Y = 4;
constexpr int BLOCK = 256;

struct Tiling {
    int n, dim, count;
    const int *mask;  // optional: fields whose mask is 0 are skipped
    int noremap = 0;  // 1: keep the hardware workgroup order (no XCD grouping)
};

__host__ __device__ inline long tiles_per_field(int n, int dim)
{
    if (dim == 3) return (long)((n + TILE_X - 1) / TILE_X) * ((n + TILE_Y - 1) / TILE_Y) * n;
    return (n + BLOCK - 1) / BLOCK;
}

__host__ inline long grid_blocks(const Tiling &t) { return tiles_per_field(t.n, t.dim) * t.count; }

__device__ inline unsigned xcd_remap(unsigned bid, unsigned nb)
{
    unsigned full = nb & ~7u;
    if (bid >= full) return bid;
    unsigned per = full >> 3;
    return (bid & 7u) * per + (bid >> 3);
}

// Decode this thread's point.  Returns false when the thread is outside the
// interior or its field is masked off.  i, j, k are 1-based interior
// indices; `off` the element offset inside the field.
template <int DIM>
__device__ inline bool tile_point(const Tiling &t, int &item, int &i, int &j, int &k, long &off)
{
    const unsigned bid = t.noremap ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const int n = t.n;
    if (DIM == 3) {
        const unsigned gx = (n + TILE_X - 1) / TILE_X, gy = (n + TILE_Y - 1) / TILE_Y;
        const unsigned per_plane = gx * gy;
        const unsigned per_field = per_plane * (unsigned)n;
        item = (int)(bid / per_field);
        unsigned rem = bid - (unsigned)item * per_field;
        k = (int)(rem / per_plane) + 1;
        rem -= (unsigned)(k - 1) * per_plane;
        const unsigned jt = rem / gx, it = rem - jt * gx;
        i = (int)(it * TILE_X + (threadIdx.x & (TILE_X - 1))) + 1;
        j = (int)(jt * TILE_Y + (threadIdx.x >> 6)) + 1;
        off = (long)i + (long)j * row_stride(n) + (long)k * plane_stride(n);
    } else {
        const unsigned per_field = (n + BLOCK - 1) / BLOCK;
        item = (int)(bid / per_field);
        const unsigned rem = bid - (unsigned)item * per_field;
        i = (int)(rem * BLOCK + threadIdx.x) + 1;
        j = k = 1;
        off = i;
    }
    if (item >= t.count) return false;
    if (t.mask && !t.mask[item]) return false;
    return i <= n && j <= n && k <= n;
}

// Column tiling for 3D streaming stencils: a thread owns one (i, j) column
// and KZ consecutive planes k0 .. k0+nk-1 (nk = KZ except at the top).  All
// loads of the KZ points are issued before any store, so each wavefront keeps
// several KB in flight; one point per thread leaves the HBM pipe latency-bound.
__host__ __device__ inline long col_tiles_per_field(int n, int kz)
{
    return (long)((n + TILE_X - 1) / TILE_X) * ((n + TILE_Y - 1) / TILE_Y) * ((n + kz - 1) / kz);
}

template <int KZ>
__device__ inline bool tile_col(const Tiling &t, int &item, int &i, int &j, int &k0, int &nk, long &off)
{
    const unsigned bid = t.noremap ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const int n = t.n;
    const unsigned gx = (n + TILE_X - 1) / TILE_X, gy = (n + TILE_Y - 1) / TILE_Y, gz = (n + KZ - 1) / KZ;
    const unsigned per_plane = gx * gy;
    const unsigned per_field = per_plane * gz;
    item = (int)(bid / per_field);
    unsigned rem = bid - (unsigned)item * per_field;
    const int kc = (int)(rem / per_plane);
    rem -= (unsigned)kc * per_plane;
    const unsigned jt = rem / gx, it = rem - jt * gx;
    i = (int)(it * TILE_X + (threadIdx.x & (TILE_X - 1))) + 1;
    j = (int)(jt * TILE_Y + (threadIdx.x >> 6)) + 1;
    k0 = kc * KZ + 1;
    nk = n - k0 + 1 < KZ ? n - k0 + 1 : KZ;
    off = (long)i + (long)j * row_stride(n) + (long)k0 * plane_stride(n);
    if (item >= t.count) return false;
    if (t.mask && !t.mask[item]) return false;
    return i <= n && j <= n;
}

// Sum over dimensions of the 3-point second differences (not divided by h^2).
template <int DIM, typename T>
__device__ inline T d2sum(const T *__restrict__ u, long c, long sy, long sz)
{
    const T uc = u[c];
    T s = u[c - 1] + u[c + 1];
    if (DIM == 3) s += (u[c - sy] + u[c + sy]) + (u[c - sz] + u[c + sz]);
    return s - (T)(2 * DIM) * uc;
}

}  // namespace pfmg
