// Host-side solver state of one pfmg context.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/pfmg.h"
#include "kernels.h"

namespace pfmg {

// Work arrays of one multigrid level for up to `cap` simultaneous solves.
struct MGLevel {
    int n = 0;
    long fs64 = 0, fs32 = 0;          // slot strides (elements)
    View<double> e{}, b{}, r{}, t{};  // levels >= 1 use e, b; r/t when needed
    View<float> e32{}, b32{}, r32{}, t32{};
};

// One PFASST level: grid, nodes, state of all slices, and its MG hierarchy.
struct PLevel {
    int n = 0, nn = 0;
    long fs = 0;                      // FP64 slot stride
    double *U = nullptr, *F = nullptr, *I = nullptr, *B = nullptr;
    double *Tau = nullptr, *Uold = nullptr, *DC = nullptr;   // coarse level only
    double *Fold = nullptr;           // coarse F at restriction (f_interp)
    double *DCF = nullptr;            // interpolated coarse F change (f_interp)
    double *Ft = nullptr;             // fine F(U) for the residual (f_solve or f_interp)
    std::vector<MGLevel> mg;          // mg[0].n == n
    long double s_ld[16];
    double s[16], Q[256], S[256], d[16];
    double *dQ = nullptr, *dS = nullptr;
    double *slot(double *base, int p, int m) const { return base + ((long)p * nn + m) * fs; }
};

struct UNet;

// Launch timing for one kernel family: brackets nest (a whole V-cycle
// contains its smoother launches); only the bracket whose family matches
// the enabled key records events, and its stop is the one at the same
// nesting depth.  A stamped bracket covers exactly one launch made through
// launch(): its events are stamped by that dispatch itself; if no such
// launch consumed them (an empty launch), the bracket is dropped.
struct Timer {
    std::string key;                  // kernel family "@" grid n, e.g. "rbgs@127"
    bool on = false;
    std::vector<hipEvent_t> ev;       // start/stop pairs
    size_t used = 0;
    int depth = 0;                    // current bracket nesting
    int open = -1;                    // depth of the recording bracket, -1 if none
    bool stamped = false;             // open bracket's events stamped by its launch
    double added = 0;                 // bytes the open bracket added
    double bytes = 0;
    long long launches = 0;
    void start(const char *fam, int n, double bytes_per_point, long points, bool stamped_launch, hipStream_t s);
    void stop(hipStream_t s);
    hipError_t enable(const char *kernel, bool enable);          // resets the counters
    hipError_t read(long long *nl, double *ms, double *nbytes);  // stream already synchronised
    void release();
};

struct Solver {
    pfmg_params p{};
    hipStream_t s = nullptr;
    int dim = 3, P = 1, nl = 1;
    PLevel L[3];                      // fine, (middle,) coarse
    double *ublock = nullptr, *ublock_c = nullptr, *fublock_c = nullptr;   // fine; coarsest level
    double *ublock_m = nullptr;               // middle level (three levels)
    double *vb = nullptr, *vu = nullptr;      // pfmg_vcycle staging slots (fine)
    double *esnap = nullptr;                  // AFTER_SWEEP: fine end values after the fine sweep [P]
    double *dLt[2] = {nullptr, nullptr};      // level l node x level l+1 node
    int cmap[2][16] = {};
    unsigned long long *bits = nullptr;       // reduction scratch [4 * P]
    int *mask = nullptr;                      // [P]
    unsigned long long *hbits = nullptr;      // pinned host mirror [4 * P]
    int *hmask = nullptr;                     // pinned host mask [P]
    bool has_state = false;
    long long vcount[3] = {0, 0, 0};
    int last_solve_status = 0;
    Timer timer;

    // --- setup
    static bool validate(const pfmg_params &p, std::string &why);
    // levels of a context (1, 2 or 3) and the node count of level lev
    static int levels(const pfmg_params &p) { return p.nodes_coarse == 0 ? 1 : p.nodes_middle > 0 ? 3 : 2; }
    static int level_nodes(const pfmg_params &p, int lev)
    {
        return lev == 0 ? p.nodes_fine : (levels(p) == 3 && lev == 1) ? p.nodes_middle : p.nodes_coarse;
    }
    static size_t carve(const pfmg_params &p, char *base, Solver *sv);   // returns bytes
    // Only what a fine-grid solve needs (one field): the multigrid
    // hierarchy of level 0, the b / u staging slots and the reduction
    // scratch.  Returns bytes (a multiple of 256).
    static size_t carve_vcycle(const pfmg_params &p, char *base, Solver *sv);
    bool init_host(std::string &why);
    hipError_t upload_constants();

    // --- building blocks (all enqueue on s)
    hipError_t solve(int lev, View<double> u, View<double> b, int count, double alpha, int cycles,
                     double *relres_host);
    hipError_t vcycle64(int lev, int l, View<double> u, View<double> b, int count, const int *mask,
                        double alpha);
    hipError_t vcycle32(int lev, int l, View<float> u, View<float> b, int count, const int *mask,
                        double alpha);
    template <typename T>
    hipError_t smooth(int n, int count, const int *mask, double alpha, View<T> u, View<T> b, View<T> tmp,
                      int sweeps, bool from_zero);
    hipError_t cycle_step(int lev, View<double> u, View<double> b, int count, const int *mask, double alpha);
    // Fourth-order fine level: the top of the V-cycle with L4, smoothing
    // passes, the residual max-norm and F of a level's operator.
    hipError_t vcycle4(int lev, View<double> u, View<double> b, int count, const int *mask, double alpha);
    hipError_t smooth4(const Tiling &t, double alpha, View<double> u, View<double> b, View<double> tmp, int sweeps);
    hipError_t resid_norm_lev(int lev, const Tiling &t, double alpha, View<double> b, View<double> u,
                              unsigned long long *out);
    hipError_t apply_F(int lev, const Tiling &t, View<double> u, View<double> F);
    // u0src / f0src (stride: one slice's node stack): node 0 of each swept
    // slice is first copied from there, in the sweep's first kernel.
    hipError_t sweep(int lev, int p0, int p1, const double *u0src = nullptr, const double *f0src = nullptr,
                     long src_stride = 0);
    // level l -> l+1 and l+1 -> l
    hipError_t fas_restrict(int p0, int p1, int l = 0);
    hipError_t interpolate(int p0, int p1, int l = 0);
    hipError_t predictor();
    hipError_t spread(const double *u0_dev);
    hipError_t residual(double *per_slice, double *block);
    hipError_t iterate(double *block);

    int noremap = 0;
    bool tune = true;                 // false: fixed launch shapes, no tuner timing runs
    bool use_bottom = true;           // small grids: whole V-cycle in one LDS kernel
    bool graphs = true;               // replay captured graphs of block start / iteration
    long fused_min_points = 2000000;  // one-pass red-black sweep from this batch size up
    hipStream_t cap = nullptr;        // private capture stream
    hipGraphExec_t g_iter = nullptr, g_start = nullptr;
    bool warm_iter = false, warm_start = false;   // first call ran eagerly
    bool use_graph() const { return graphs && p.vcycles_per_solve > 0 && !timer.on; }
    long long vc_iter[3] = {0, 0, 0}, vc_start[3] = {0, 0, 0};   // V-cycles of one replay
    // learned initial guess and the recording of training pairs
    UNet *unet = nullptr;
    double *nnsc = nullptr, *hnnsc = nullptr;   // per-field scale factors [2P], device and pinned host
    __bf16 *rec_pairs = nullptr;
    float *rec_ah2 = nullptr;
    double *rec_scratch = nullptr;
    int rec_cap = 0, rec_count = 0;
    long long guess_tried = 0, guess_taken = 0;
    hipError_t learned_guess(View<double> u, View<double> b, int count, double alpha, const std::vector<double> &nb,
                             std::vector<double> &rold, bool rec);
    hipError_t capture(const std::function<hipError_t()> &fn, hipGraphExec_t *out, long long *vc);
    void release_graphs();
    hipError_t spread_body();
    hipError_t iterate_body();
    hipError_t residual_enqueue();
    hipError_t snapshot_ends(int p0, int p1);
    hipError_t residual_slices(int p0, int p1);
    hipError_t chain_step(int q);
    hipError_t iterate_pipelined();
    static constexpr int MAXGROUPS = 16;
    int groups = 1;                   // slice groups of the pipelined iteration
    std::vector<int> gbound;          // group g holds slices gbound[g] .. gbound[g+1]-1
    hipStream_t s2 = nullptr;         // coarse-chain stream of the pipelined iteration
    hipEvent_t ev[MAXGROUPS + 1] = {};
    hipStream_t s3 = nullptr;         // second fine-sweep stream of the pipelined iteration
    hipEvent_t ev_fork = nullptr;
    hipEvent_t evc[2] = {};           // coarse chain done through group G-2 / G-1
    int fine_streams = 1;             // streams the groups' fine sweeps alternate over
    bool late_interp = true;          // interpolation and residual of the early groups under the last chain
    bool one_stream = false;          // the chain on the main stream too (no overlap)
    bool fused_sdc = true;            // sdc_start and apply_L_rhs in place of their separate kernels
    int mg_off = 0;                   // first multigrid scratch field of the current sweep
    template <typename T>
    View<T> scr(View<T> v) const { return View<T>{v.p ? v.p + (long)mg_off * v.stride : nullptr, v.stride}; }
    hipError_t residual_read(double *per_slice, double *block);
    Tiling tl(int n, int count, const int *m = nullptr) const { return Tiling{n, dim, count, m, noremap}; }
    void tstart(const char *fam, int n, double bytes_per_point, long points, bool stamped = false);
    void tstop();
};

}  // namespace pfmg
