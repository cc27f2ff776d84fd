// Point-per-thread tiling shared by the grid kernels.
//
// A launch covers `count` fields of one grid, or up to MAXSEG segments of
// fields of different grids (the uneven problems of a batch advance in one
// launch per multigrid level): segment s has its own n, field count, mask
// and per-field scalar (the kernel's alpha, delta, nu or dt), and every View
// its own base and stride per segment.  The workgroups of the segments
// follow each other in launch order.  3D: a workgroup of 256
// threads (4 wavefronts) owns a 64 x 4 patch of one z-plane of one field,
// one wavefront per 64-point row segment, so every wavefront reads and
// writes whole 512-byte (FP64) row segments.  1D: 256 consecutive points.
//
// The flat workgroup id is remapped so that each of the 8 XCDs (which
// receive workgroups round-robin) gets one contiguous run of tiles: the
// planes k-1, k, k+1 of a tile and the neighbouring rows then mostly meet
// in the same XCD's L2.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "layout.h"

namespace pfmg {

constexpr int TILE_X = 64;
constexpr int TILE_Y = 4;
constexpr int BLOCK = 256;

constexpr int MAXSEG = 4;

struct SegX {
    int n, count;
    const int *mask;
    const double *coef;
};

struct Tiling {
    int n, dim, count;              // segment 0
    const int *mask;                // optional: fields whose mask is 0 are skipped
    int noremap = 0;                // 1: keep the hardware workgroup order (no XCD grouping)
    const double *coef = nullptr;   // optional per-field scalar of segment 0
    int nseg = 1;
    SegX x[MAXSEG - 1] = {};        // segments 1 .. nseg-1
    __host__ __device__ int seg_n(int s) const { return s == 0 ? n : x[s - 1].n; }
    __host__ __device__ int seg_count(int s) const { return s == 0 ? count : x[s - 1].count; }
};

// Where a workgroup landed: segment, field, grid size, per-field scalar.
struct Pt {
    int sg, item, n;
    const double *coef;
    __device__ double par(double x) const { return coef ? coef[item] : x; }
};

// Find the segment of local workgroup id `bid` (made segment-relative);
// per_field(n) is the launch's workgroups per field.
template <class PF>
__host__ __device__ inline bool find_seg(const Tiling &t, unsigned &bid, Pt &q, const int *&mask, PF per_field)
{
    q.sg = 0;
    q.n = t.n;
    q.coef = t.coef;
    mask = t.mask;
    unsigned tiles = (unsigned)(per_field(t.n) * t.count);
    for (int s = 1; s < t.nseg && bid >= tiles; ++s) {
        bid -= tiles;
        q.sg = s;
        q.n = t.x[s - 1].n;
        q.coef = t.x[s - 1].coef;
        mask = t.x[s - 1].mask;
        tiles = (unsigned)(per_field(q.n) * t.x[s - 1].count);
    }
    return bid < tiles;
}

template <class PF>
__host__ inline long total_blocks(const Tiling &t, PF per_field)
{
    long b = 0;
    for (int s = 0; s < t.nseg; ++s) b += per_field(t.seg_n(s)) * t.seg_count(s);
    return b;
}

__host__ __device__ inline long tiles_per_field(int n, int dim)
{
    if (dim == 3) return (long)((n + TILE_X - 1) / TILE_X) * ((n + TILE_Y - 1) / TILE_Y) * n;
    return (n + BLOCK - 1) / BLOCK;
}

__host__ inline long grid_blocks(const Tiling &t)
{
    const int dim = t.dim;
    return total_blocks(t, [dim](int n) { return tiles_per_field(n, dim); });
}

template <typename T>
__device__ inline T *fp(const View<T> &v, const Pt &q)
{
    return q.sg == 0 ? v.p + (long)q.item * v.stride : v.px[q.sg - 1] + (long)q.item * v.sx[q.sg - 1];
}

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
__device__ inline bool tile_point(const Tiling &t, Pt &q, int &i, int &j, int &k, long &off)
{
    unsigned bid = t.noremap ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const int *mask;
    if (!find_seg(t, bid, q, mask, [](int n) { return tiles_per_field(n, DIM); })) return false;
    const int n = q.n;
    if (DIM == 3) {
        const unsigned gx = (n + TILE_X - 1) / TILE_X, gy = (n + TILE_Y - 1) / TILE_Y;
        const unsigned per_plane = gx * gy;
        const unsigned per_field = per_plane * (unsigned)n;
        q.item = (int)(bid / per_field);
        unsigned rem = bid - (unsigned)q.item * per_field;
        k = (int)(rem / per_plane) + 1;
        rem -= (unsigned)(k - 1) * per_plane;
        const unsigned jt = rem / gx, it = rem - jt * gx;
        i = (int)(it * TILE_X + (threadIdx.x & (TILE_X - 1))) + 1;
        j = (int)(jt * TILE_Y + (threadIdx.x >> 6)) + 1;
        off = (long)i + (long)j * row_stride(n) + (long)k * plane_stride(n);
    } else {
        const unsigned per_field = (n + BLOCK - 1) / BLOCK;
        q.item = (int)(bid / per_field);
        const unsigned rem = bid - (unsigned)q.item * per_field;
        i = (int)(rem * BLOCK + threadIdx.x) + 1;
        j = k = 1;
        off = i;
    }
    if (mask && !mask[q.item]) return false;
    return i <= n && j <= n && k <= n;
}

// The field a workgroup of a point-tiled launch belongs to (all its threads
// share it), or -1 past the end.
template <int DIM>
__device__ inline bool tile_block_item(const Tiling &t, Pt &q)
{
    unsigned bid = t.noremap ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const int *mask;
    if (!find_seg(t, bid, q, mask, [](int n) { return tiles_per_field(n, DIM); })) return false;
    q.item = (int)(bid / (unsigned)tiles_per_field(q.n, DIM));
    return true;
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
__device__ inline bool tile_col(const Tiling &t, Pt &q, int &i, int &j, int &k0, int &nk, long &off)
{
    unsigned bid = t.noremap ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const int *mask;
    if (!find_seg(t, bid, q, mask, [](int n) { return col_tiles_per_field(n, KZ); })) return false;
    const int n = q.n;
    const unsigned gx = (n + TILE_X - 1) / TILE_X, gy = (n + TILE_Y - 1) / TILE_Y, gz = (n + KZ - 1) / KZ;
    const unsigned per_plane = gx * gy;
    const unsigned per_field = per_plane * gz;
    q.item = (int)(bid / per_field);
    unsigned rem = bid - (unsigned)q.item * per_field;
    const int kc = (int)(rem / per_plane);
    rem -= (unsigned)kc * per_plane;
    const unsigned jt = rem / gx, it = rem - jt * gx;
    i = (int)(it * TILE_X + (threadIdx.x & (TILE_X - 1))) + 1;
    j = (int)(jt * TILE_Y + (threadIdx.x >> 6)) + 1;
    k0 = kc * KZ + 1;
    nk = n - k0 + 1 < KZ ? n - k0 + 1 : KZ;
    off = (long)i + (long)j * row_stride(n) + (long)k0 * plane_stride(n);
    if (mask && !mask[q.item]) return false;
    return i <= n && j <= n;
}

template <int KZ>
__host__ inline long col_blocks(const Tiling &t)
{
    return total_blocks(t, [](int n) { return col_tiles_per_field(n, KZ); });
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

// ------------------------------------------------------- stamped launches
// Kernel timing without marker packets: the host arms a start/stop event
// pair, and the next launch made through launch() hands both to
// hipExtLaunchKernel, which stamps them with that dispatch's own begin and
// end.  An event recorded between host launches would also count the time
// the queue sits idle while the host issues the kernel.  Unarmed launches
// are plain hipLaunchKernel calls.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
inline thread_local LaunchEvents armed_events;

template <typename T>
struct same_type {
    using type = T;
};

template <typename... P>
__host__ inline hipError_t launch(void (*kernel)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s,
                                  typename same_type<P>::type... a)
{
    void *argv[] = {(void *)&a..., nullptr};
    if (armed_events.start) {
        const LaunchEvents e = armed_events;
        armed_events = {};
        return hipExtLaunchKernel((const void *)kernel, grid, block, argv, lds, s, e.start, e.stop, 0);
    }
    return hipLaunchKernel((const void *)kernel, grid, block, argv, lds, s);
}

}  // namespace pfmg
