// Launch-shape autotuner for the red-black smoother.
//
// A red-black sweep over a batch of 3D grids can run as two colour passes
// (point-tiled, in place) or as the one-pass out-of-place kernel with a
// choice of rows per workgroup (ty) and planes per z-chunk.  Which is
// fastest depends on the grids, the number of fields and the precision: the
// one-pass kernel streams its z-chunks serially, so few small fields favour
// the colour passes.  The tuner times the candidates on the launch's own
// buffers the first time a configuration is met outside graph capture and
// keeps the winner for the process; with PFMG_TUNE_CACHE=<file> the table is
// also read from and appended to that file.  Keys name the device, kernel,
// precision and every segment's n x field count, e.g.
// "gfx950/rbgs/f64/127x16+63x32".  PFMG_TUNE=0 turns timing off (the
// defaults below are used instead).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "kernels.h"

namespace pfmg {

struct RbPlan {
    bool fused = false;
    k::FusedShape shape{};
};

// Plan for `sweeps` red-black sweeps of the launch `t` (3D, every n in
// 31..255, a ping-pong buffer available).  May launch timing runs of both
// variants on `s` that write only `tmp`.  fallback_fused: the choice when
// no timing is allowed (stream capture, PFMG_TUNE=0).
template <typename T>
RbPlan rb_plan(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, View<T> tmp, hipStream_t s,
               bool fallback_fused);

// Number of configurations tuned or loaded so far (for tests and reports).
int tune_table_size();
// The entry for a key ("" if none), as "fused ty zchunk blocks" (fused: 0
// colour passes, 1 one-pass kernel with 256-thread workgroups, 2 with 512).
std::string tune_lookup(const std::string &key);
// Pins the entry for a key, replacing any timed or loaded one (not written
// to the cache file); fused = -1 drops the entry.  False for a malformed key
// or a one-pass shape the kernel is not instantiated for.
bool tune_set(const std::string &key, int fused, int ty, int zchunk);

}  // namespace pfmg
