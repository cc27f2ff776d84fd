// Device data layout of one grid function (interior n^dim points plus a
// one-point zero halo carrying the homogeneous Dirichlet data).
//
// 3D: element (i,j,k), i,j,k in [0, n+1], sits at i + j*sy + k*sz with
//     sy = n+1 and sz = (n+1)(n+2).  The right halo point of row j
//     (i = n+1) is the same memory as the left halo point of row j+1
//     (i = 0); both are zero, so one halo word per row suffices.  For the
//     usual n = 2^q - 1 a row is then exactly 2^q words, so every interior
//     row starts on a 256-byte boundary once element 1 does.
// 1D: element i in [0, n+1] sits at i.
// Element count: (n+1)(n+2)^2 + 1 in 3D, n+2 in 1D.  Each field occupies a
// slot of `field_stride` elements: 256 bytes of lead so that element 1 is
// 256-byte aligned, then the elements, rounded up to 256 bytes.  The halo
// words are zeroed once (the workspace is cleared at creation) and never
// written by any kernel.
#pragma once
#include <cstddef>
#include <cstdint>

#ifndef PFMG_HD
#if defined(__HIPCC__)
#define PFMG_HD __host__ __device__
#else
#define PFMG_HD
#endif
#endif

namespace pfmg {

PFMG_HD inline long row_stride(int n) { return (long)n + 1; }
PFMG_HD inline long plane_stride(int n) { return ((long)n + 1) * ((long)n + 2); }

PFMG_HD inline long field_elems(int n, int dim)
{
    return dim == 3 ? ((long)n + 1) * ((long)n + 2) * ((long)n + 2) + 1 : (long)n + 2;
}

// Offset of element 0 inside a slot: element 1 lands 256 bytes in.
PFMG_HD inline long field_lead(size_t elem_bytes) { return (long)(256 / elem_bytes) - 1; }

PFMG_HD inline long field_stride(int n, int dim, size_t elem_bytes)
{
    size_t bytes = 256 + (size_t)field_elems(n, dim) * elem_bytes;
    bytes = (bytes + 255) / 256 * 256;
    return (long)(bytes / elem_bytes);
}

// The nodes of one slice (and the slices of a level) sit in consecutive
// slots, so the distance between node m and m+1 of a grid is its slot stride.
PFMG_HD inline long node_stride(int n, int dim) { return field_stride(n, dim, sizeof(double)); }

PFMG_HD inline long interior_points(int n, int dim)
{
    return dim == 3 ? (long)n * n * n : (long)n;
}

// Next-coarser multigrid grid: coarse point J (1-based) sits on fine 2J.
PFMG_HD inline int coarser(int n) { return (n + 1) / 2 - 1; }

// A batch of `count` fields of one grid, field q at p + q * stride
// (p already points at element 0 of field 0).
// Segments 1..3 of a multi-segment launch keep their bases in px / sx.
template <typename T>
struct View {
    T *p;
    long stride;
    T *px[3] = {nullptr, nullptr, nullptr};
    long sx[3] = {0, 0, 0};
};

}  // namespace pfmg
