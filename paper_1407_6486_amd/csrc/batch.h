// Batched IPFASST: many independent heat problems, each with its own grid
// size, nu and dt, advanced together.  Problems of one grid size form a
// group; every launch covers all groups (up to MAXSEG segments per launch),
// so one launch per multigrid level and leg serves every (problem, slice)
// pair that has that level.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/pfmg.h"
#include "kernels.h"
#include "solver.h"

namespace pfmg {

// One size group.  Items are (problem, slice) pairs, problem-major with the
// slice fastest: item = q * P + p for the group's q-th problem.
struct BGroup {
    int n = 0, nprob = 0, items = 0, item0 = 0;   // item0: first flat item over all groups
    std::vector<int> probs;                        // problem ids of the group, in order
    PLevel L[2];                                   // state of all items, MG arrays for `items` fields
    double *ublock = nullptr, *ublock_c = nullptr, *fublock_c = nullptr;   // one slot per problem
    // Offsets of the group's tables.  Per-field scalars (in `coef`): _i per
    // item, _p per problem, nu_f per (item, node) field; alpha = nu dt d[m]
    // and delta = dt d[m] per node m >= 1 of each level.
    long o_dt_i = 0, o_dt_p = 0, o_nu_i = 0, o_nu_p = 0, o_nu_f[2] = {0, 0};
    long o_alpha_i[2][16] = {}, o_delta_i[2][16] = {}, o_alpha_p[2][16] = {}, o_delta_p[2][16] = {};
    // Fixed masks (in `fixed_mask`): from[j][item] = item % P >= j;
    // shift[j][i] = (i + 1) % P >= max(j, 1) for the copy of item i's end
    // value into item i + 1.
    long o_from = 0, o_shift = 0;
    // Masks of the problems still iterating (in `act`): per item, per
    // problem, per (item, node) field of each level, per shifted copy.
    long o_act_i = 0, o_act_p = 0, o_act_f[2] = {0, 0}, o_act_shift = 0;
};

// One group's operands of a multigrid solve at one depth.
template <typename T>
struct Leg {
    int g, lev, d, n, count;
    const int *mask;
    const double *alpha;
    View<T> u, b, t;
};

struct BatchSolver {
    pfmg_params p{};                   // shared method parameters
    std::vector<pfmg_params> prob;     // per problem (n, nu, dt differ)
    hipStream_t s = nullptr;
    int dim = 3, P = 1, nl = 2, NP = 0, ng = 0, total_items = 0;
    std::vector<BGroup> G;
    std::vector<int> grp_of, loc_of;   // problem -> group, index inside the group
    int nn[2] = {0, 0};
    long double s_ld[2][16];
    double Q[2][256], S[2][256], d[2][16];
    double *dQ[2] = {nullptr, nullptr}, *dS[2] = {nullptr, nullptr}, *dLt = nullptr;
    int cmap[16] = {0};
    double *stage = nullptr;           // one dense array of the largest grid
    unsigned long long *bits = nullptr, *hbits = nullptr;   // [2][total_items][RSLOTS]
    double *coef = nullptr;            // device tables of per-field scalars
    int *fixed_mask = nullptr;
    int *act = nullptr, *hact = nullptr;   // active masks, device and pinned host mirror
    std::vector<double> coef_host;
    std::vector<int> fixed_host, act_init;
    std::vector<char> active;          // per problem
    std::vector<double> res;           // per problem: last residual
    std::vector<int> iters;            // per problem: iterations run in this block
    bool act_dirty = true;
    bool has_state = false, use_bottom = true, graphs = true, nan = false;
    int noremap = 0;
    long fused_min_points = 2000000;
    long long vcount[2] = {0, 0};
    hipStream_t cap = nullptr;
    hipGraphExec_t g_iter = nullptr, g_start = nullptr;
    bool warm_iter = false, warm_start = false;
    Timer timer;                       // launch timing (blocks run eagerly while on)
    bool use_graph() const { return graphs && !timer.on; }

    static bool validate(const pfmg_params *pp, int np, std::string &why);
    bool init_host(const pfmg_params *pp, int np, std::string &why);   // groups, tables
    size_t carve(char *base);                                          // workspace layout
    hipError_t upload();                                               // constants, tables, masks

    // building blocks (enqueue on s)
    const double *C(long o) const { return coef + o; }
    const int *FM(long o) const { return fixed_mask + o; }
    const int *AM(long o) const { return act + o; }
    template <typename T, class Fn>
    hipError_t chunks(const std::vector<Leg<T>> &v, Fn fn) const;
    template <typename T>
    hipError_t vcycle(std::vector<Leg<T>> top, bool zero_top);
    template <typename T>
    hipError_t smooth(const std::vector<Leg<T>> &legs, int sweeps, bool from_zero);
    hipError_t cycle_step(const std::vector<Leg<double>> &top);
    hipError_t sweep(int lev, int chain, bool masked_round, int round);
    hipError_t fas_restrict(bool masked);
    hipError_t interpolate(bool masked);
    hipError_t spread_body();
    hipError_t iterate_body();
    hipError_t set_initial(const double *u0, bool on_device);
    hipError_t iterate();
    void freeze(int problem);
    hipError_t get(int problem, int field, int slice, int node, double *dst, bool on_device);
    hipError_t capture(const std::function<hipError_t()> &fn, hipGraphExec_t *out);
    void release();
};

}  // namespace pfmg
