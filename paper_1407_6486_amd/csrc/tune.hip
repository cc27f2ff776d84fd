// Launch-shape autotuner for the red-black smoother (see tune.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "tune.h"

namespace pfmg {
namespace {

struct Entry {
    int fused, ty, zchunk;
    long blocks;
};

std::mutex g_mu;
std::map<std::string, Entry> g_table;
bool g_loaded = false;

const char *cache_path()
{
    const char *e = getenv("PFMG_TUNE_CACHE");
    return e && *e ? e : nullptr;
}

void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[512];
    Entry e;
    while (fscanf(f, "%511s %d %d %d %ld", key, &e.fused, &e.ty, &e.zchunk, &e.blocks) == 5) g_table[key] = e;
    fclose(f);
}

void append_locked(const std::string &key, const Entry &e)
{
    const char *path = cache_path();
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %ld\n", key.c_str(), e.fused, e.ty, e.zchunk, e.blocks);
    fclose(f);
}

// PFMG_TUNE_VERBOSE=1: every timed candidate is reported on stderr.
bool verbose()
{
    static const bool v = [] {
        const char *e = getenv("PFMG_TUNE_VERBOSE");
        return e && atoi(e) != 0;
    }();
    return v;
}

bool tuning_enabled()
{
    const char *e = getenv("PFMG_TUNE");
    return !(e && atoi(e) == 0);
}

template <typename T>
std::string make_key(const Tiling &t)
{
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    }
    std::string key = arch + "/rbgs/" + (sizeof(T) == 8 ? "f64/" : "f32/");
    for (int sg = 0; sg < t.nseg; ++sg) {
        if (sg) key += "+";
        key += std::to_string(t.seg_n(sg)) + "x" + std::to_string(t.seg_count(sg));
    }
    return key;
}

// Average milliseconds of `reps` runs of fn after one warm-up run.
template <class F>
float time_ms(F fn, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps)
{
    if (fn() != hipSuccess) return -1.f;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r)
        if (fn() != hipSuccess) return -1.f;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
    return ms / reps;
}

}  // namespace

template <typename T>
RbPlan rb_plan(const Tiling &t, double alpha, double omega, View<T> b, View<T> u, View<T> tmp, hipStream_t s,
               bool fallback_fused)
{
    RbPlan plan;
    const std::string key = make_key<T>(t);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_locked();
        auto it = g_table.find(key);
        if (it != g_table.end()) {
            const Entry &e = it->second;
            plan.fused = e.fused != 0;
            if (plan.fused) {
                // fused = 2: 512-thread workgroups
                plan.shape = k::rbgs_fused_shape(t, sizeof(T), e.ty, 1, e.fused == 2 ? 512 : 256);
                plan.shape.zchunk = e.zchunk;
                long blocks = 0;
                for (int sg = 0; sg < t.nseg; ++sg) {
                    const int n = t.seg_n(sg);
                    blocks += (long)t.seg_count(sg) * ((n + e.ty - 1) / e.ty) * ((n + e.zchunk - 1) / e.zchunk);
                }
                plan.shape.blocks = blocks;
                if (plan.shape.ty != e.ty || e.zchunk < 1) plan.shape = k::rbgs_fused_shape(t, sizeof(T));
            }
            return plan;
        }
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
    if (capturing || !tuning_enabled()) {
        plan.fused = fallback_fused;
        if (plan.fused) plan.shape = k::rbgs_fused_shape(t, sizeof(T));
        return plan;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        plan.fused = fallback_fused;
        if (plan.fused) plan.shape = k::rbgs_fused_shape(t, sizeof(T));
        return plan;
    }
    const int reps = 3;
    // colour passes, in place on a copy of u held in tmp
    float best = 0;
    Entry win{0, 0, 0, 0};
    if (k::copy(t, u, tmp, s) == hipSuccess) {
        best = time_ms([&] {
            hipError_t e = k::rbgs(t, alpha, omega, 0, b, tmp, s);
            return e == hipSuccess ? k::rbgs(t, alpha, omega, 1, b, tmp, s) : e;
        }, s, e0, e1, reps);
    }
    if (best < 0) best = 1e30f;
    if (verbose()) fprintf(stderr, "tune %s colour-passes %.2f us\n", key.c_str(), best * 1e3f);
    // one-pass shapes: rows per workgroup x planes per z-chunk (short
    // chunks let small grids spread over more workgroups; every chunk also
    // recomputes its two border planes)
    std::vector<k::FusedShape> cands;
    int nmax = 0;
    for (int sg = 0; sg < t.nseg; ++sg) nmax = std::max(nmax, t.seg_n(sg));
    for (int nt : {256, 512})
    for (int ty : {2, 4, 6, 8, 10, 12, 16, 22})
        for (int zc : {2, 3, 4, 6, 8, 12, 16, 24, 32, 64, 128, 256}) {
            k::FusedShape f = k::rbgs_fused_shape(t, sizeof(T), ty, 1, nt);
            if (f.ty != ty || zc > nmax) continue;
            f.zchunk = zc;
            f.blocks = 0;
            for (int sg = 0; sg < t.nseg; ++sg) {
                const int n = t.seg_n(sg);
                f.blocks += (long)t.seg_count(sg) * ((n + ty - 1) / ty) * ((n + zc - 1) / zc);
            }
            if (f.blocks <= 0 || f.blocks > 16384) continue;
            cands.push_back(f);
        }
    for (const auto &f : cands) {
        const float ms = time_ms([&] { return k::rbgs_fused(t, alpha, omega, false, b, u, tmp, s, &f); }, s, e0, e1,
                                 reps);
        if (verbose())
            fprintf(stderr, "tune %s fused nt %d ty %d zchunk %d blocks %ld %.2f us\n", key.c_str(), f.nt, f.ty,
                    f.zchunk, f.blocks, ms * 1e3f);
        if (ms >= 0 && ms < best) {
            best = ms;
            win = Entry{f.nt == 512 ? 2 : 1, f.ty, f.zchunk, f.blocks};
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipGetLastError();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[key] = win;
        append_locked(key, win);
    }
    plan.fused = win.fused != 0;
    if (plan.fused)
        for (const auto &f : cands)
            if (f.ty == win.ty && f.zchunk == win.zchunk && f.nt == (win.fused == 2 ? 512 : 256)) plan.shape = f;
    return plan;
}

int tune_table_size()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_table.size();
}

std::string tune_lookup(const std::string &key)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(key);
    if (it == g_table.end()) return "";
    const Entry &e = it->second;
    return std::to_string(e.fused) + " " + std::to_string(e.ty) + " " + std::to_string(e.zchunk) + " " +
           std::to_string(e.blocks);
}

bool tune_set(const std::string &key, int fused, int ty, int zchunk)
{
    // "<arch>/rbgs/<f64|f32>/" then n x count per segment, joined by '+'
    const size_t p0 = key.find("/rbgs/");
    if (p0 == std::string::npos || p0 == 0) return false;
    const std::string prec = key.substr(p0 + 6, 4);
    if (prec != "f64/" && prec != "f32/") return false;
    std::vector<std::pair<int, long>> segs;
    const char *c = key.c_str() + p0 + 10;
    while (true) {
        char *end = nullptr;
        const long n = strtol(c, &end, 10);
        if (end == c || *end != 'x' || n < 1 || n > 255) return false;
        c = end + 1;
        const long cnt = strtol(c, &end, 10);
        if (end == c || cnt < 1 || cnt > (1L << 20)) return false;
        segs.emplace_back((int)n, cnt);
        c = end;
        if (*c == 0) break;
        if (*c != '+') return false;
        ++c;
    }
    if (fused < -1 || fused > 2) return false;
    if (fused == -1) {
        std::lock_guard<std::mutex> lk(g_mu);
        load_locked();
        g_table.erase(key);
        return true;
    }
    Entry e{0, 0, 0, 0};
    if (fused != 0) {
        int nmax = 0;
        for (const auto &sc : segs) nmax = std::max(nmax, sc.first);
        if (zchunk < 1 || ty > nmax || !k::rbgs_fused_ty_ok(nmax, ty, fused == 2 ? 512 : 256)) return false;
        long blocks = 0;
        for (const auto &sc : segs)
            blocks += sc.second * ((sc.first + ty - 1) / ty) * ((sc.first + zchunk - 1) / zchunk);
        if (blocks > (1L << 30)) return false;
        e = Entry{fused, ty, zchunk, blocks};
    }
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_table[key] = e;
    return true;
}

template RbPlan rb_plan<double>(const Tiling &, double, double, View<double>, View<double>, View<double>, hipStream_t,
                                bool);
template RbPlan rb_plan<float>(const Tiling &, double, double, View<float>, View<float>, View<float>, hipStream_t,
                               bool);

}  // namespace pfmg
