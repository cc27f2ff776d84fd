// Batched IPFASST (see batch.h).
//
// Each problem follows the same algorithm as a single context (Sec. 2.4:
// predictor, then iterations of fine sweep, FAS restriction, coarse sweeps
// in slice order, interpolation and the collocation residual); only the
// launches are shared.  Per-problem nu and dt enter the kernels as
// per-field scalar tables, and the predictor rounds (slice p sweeps in
// rounds 0..p) and the node-0 updates (no copy across problem boundaries)
// as per-field masks.  A problem whose block residual reaches pfasst_tol is
// frozen: the masks of its fields are cleared, so later iterations leave
// its state as it was when it converged, as a single context stopping at
// the same tolerance would.
//
// Multigrid by depth: depth d is level d below each problem's own grid.
// All groups still above their bottom level at depth d smooth and restrict
// in one launch per step; every group's bottom solve (the LDS V-cycle of the
// small grids, or the exact solve of n <= 2) is one launch; the upward leg
// mirrors the downward one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "batch.h"
#include "collocation.h"
#include "tune.h"

#define HC(x)                                  \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

namespace pfmg {
namespace {

inline double bits_to_double(unsigned long long b)
{
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

// One group's part of a launch: grid, fields, mask, per-field scalar and up
// to NV field views.
constexpr int NV = 6;
struct Seg {
    int n, count;
    const int *mask;
    const double *coef;
    View<double> v[NV];
};

// Launch fn once per run of up to MAXSEG non-empty segments.  fn(t, views,
// first): `first` is the index in r of the run's first segment; the run's
// segments are consecutive in r apart from empty ones left out.
template <class Fn>
hipError_t for_segs(const std::vector<Seg> &r, int dim, int noremap, Fn fn)
{
    std::vector<Seg> q;
    std::vector<int> idx;
    for (size_t w = 0; w < r.size(); ++w)
        if (r[w].count > 0) {
            q.push_back(r[w]);
            idx.push_back((int)w);
        }
    for (size_t a = 0; a < q.size(); a += MAXSEG) {
        const int ns = (int)std::min<size_t>(MAXSEG, q.size() - a);
        const Seg &h = q[a];
        Tiling t{h.n, dim, h.count, h.mask, noremap, h.coef, ns};
        View<double> v[NV];
        for (int k = 0; k < NV; ++k) v[k] = h.v[k];
        for (int w = 1; w < ns; ++w) {
            const Seg &x = q[a + w];
            t.x[w - 1] = SegX{x.n, x.count, x.mask, x.coef};
            for (int k = 0; k < NV; ++k) {
                v[k].px[w - 1] = x.v[k].p;
                v[k].sx[w - 1] = x.v[k].stride;
            }
        }
        HC(fn(t, v, idx[a]));
    }
    return hipSuccess;
}

template <typename T, class Get>
View<T> cat(const Leg<T> *x, int ns, Get get)
{
    View<T> v = get(x[0]);
    for (int w = 1; w < ns; ++w) {
        const View<T> y = get(x[w]);
        v.px[w - 1] = y.p;
        v.sx[w - 1] = y.stride;
    }
    return v;
}

template <typename T> View<T> mg_e(const MGLevel &M);
template <typename T> View<T> mg_b(const MGLevel &M);
template <typename T> View<T> mg_t(const MGLevel &M);
template <> View<double> mg_e<double>(const MGLevel &M) { return M.e; }
template <> View<double> mg_b<double>(const MGLevel &M) { return M.b; }
template <> View<double> mg_t<double>(const MGLevel &M) { return M.t; }
template <> View<float> mg_e<float>(const MGLevel &M) { return M.e32; }
template <> View<float> mg_b<float>(const MGLevel &M) { return M.b32; }
template <> View<float> mg_t<float>(const MGLevel &M) { return M.t32; }

}  // namespace

// ------------------------------------------------------------------ setup
bool BatchSolver::validate(const pfmg_params *pp, int np, std::string &why)
{
    if (!pp || np < 1 || np > 4096) { why = "n_problems must be in 1..4096"; return false; }
    const pfmg_params &a = pp[0];
    for (int q = 0; q < np; ++q) {
        const pfmg_params &b = pp[q];
        if (!Solver::validate(b, why)) { why = "problem " + std::to_string(q) + ": " + why; return false; }
        const bool same = a.dim == b.dim && a.n_slices == b.n_slices && a.nodes_fine == b.nodes_fine &&
                          a.nodes_coarse == b.nodes_coarse && a.node_family == b.node_family &&
                          a.smoother == b.smoother && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post &&
                          a.omega == b.omega && a.vcycles_per_solve == b.vcycles_per_solve &&
                          a.precision == b.precision && a.guess == b.guess && a.fine_send == b.fine_send &&
                          a.pfasst_tol == b.pfasst_tol && a.pfasst_max_iter == b.pfasst_max_iter;
        if (!same) {
            why = "problem " + std::to_string(q) + " differs from problem 0 in a method parameter (only n, nu and dt may differ)";
            return false;
        }
    }
    if (a.vcycles_per_solve < 1) { why = "batched node solves take a fixed number of V-cycles (vcycles_per_solve >= 1)"; return false; }
    if (a.fine_send != PFMG_SEND_AFTER_ITER) { why = "a batch sends the fine end value after the iteration (PFMG_SEND_AFTER_ITER)"; return false; }
    if (a.n_slices > 64) { why = "a batch takes at most 64 slices per problem"; return false; }
    if (a.stencil_order != 2 || a.interp_order != 2) {
        why = "a batch runs the second-order stencil and d-linear interpolation"; return false;
    }
    if (a.f_solve != 0 || a.f_interp != 0) {
        why = "a batch re-evaluates F (f_solve = f_interp = 0)"; return false;
    }
    if (a.residual_abs != 0) { why = "a batch uses the relative residual (residual_abs = 0)"; return false; }
    if (a.nodes_middle != 0) { why = "a batch runs one or two levels (nodes_middle = 0)"; return false; }
    return true;
}

bool BatchSolver::init_host(const pfmg_params *pp, int np, std::string &why)
{
    const char *e = getenv("PFMG_NO_XCD_REMAP");
    noremap = (e && atoi(e)) ? 1 : 0;
    e = getenv("PFMG_NO_BOTTOM");
    use_bottom = !(e && atoi(e));
    e = getenv("PFMG_NO_GRAPH");
    graphs = !(e && atoi(e));
    e = getenv("PFMG_FUSED_MIN");
    fused_min_points = e ? atol(e) : 2000000;
    p = pp[0];
    prob.assign(pp, pp + np);
    NP = np;
    dim = p.dim;
    P = p.n_slices;
    nl = p.nodes_coarse > 0 ? 2 : 1;
    nn[0] = p.nodes_fine;
    nn[1] = p.nodes_coarse;
    // groups by grid size, largest first
    std::vector<int> sizes;
    for (int q = 0; q < np; ++q)
        if (std::find(sizes.begin(), sizes.end(), pp[q].n) == sizes.end()) sizes.push_back(pp[q].n);
    std::sort(sizes.begin(), sizes.end(), [](int x, int y) { return x > y; });
    ng = (int)sizes.size();
    G.assign(ng, BGroup{});
    grp_of.assign(np, 0);
    loc_of.assign(np, 0);
    for (int g = 0; g < ng; ++g) G[g].n = sizes[g];
    for (int q = 0; q < np; ++q) {
        const int g = (int)(std::find(sizes.begin(), sizes.end(), pp[q].n) - sizes.begin());
        grp_of[q] = g;
        loc_of[q] = G[g].nprob++;
        G[g].probs.push_back(q);
    }
    total_items = 0;
    for (auto &B : G) {
        B.items = B.nprob * P;
        B.item0 = total_items;
        total_items += B.items;
    }
    for (int lev = 0; lev < nl; ++lev) {
        if (!family_nodes_ld(p.node_family, nn[lev], s_ld[lev])) { why = "node construction failed"; return false; }
        if (!collocation_matrices(nn[lev], s_ld[lev], Q[lev], S[lev], d[lev], p.node_family == PFMG_NODES_UNIFORM ? 1 : 0)) {
            why = "Q construction failed"; return false;
        }
    }
    if (nl > 1)
        for (int mc = 0; mc < nn[1]; ++mc) {
            cmap[mc] = -1;
            for (int mf = 0; mf < nn[0]; ++mf)
                if (std::fabs((double)(s_ld[0][mf] - s_ld[1][mc])) < 1e-14) cmap[mc] = mf;
            if (cmap[mc] < 0) { why = "coarse nodes must be a subset of the fine nodes"; return false; }
        }
    // tables: values exactly as a single context forms them (delta = dt d,
    // alpha = nu delta)
    coef_host.clear();
    fixed_host.clear();
    act_init.clear();
    auto addd = [&](long len) { const long o = (long)coef_host.size(); coef_host.resize(o + len, 0.0); return o; };
    auto addf = [&](long len) { const long o = (long)fixed_host.size(); fixed_host.resize(o + len, 0); return o; };
    auto adda = [&](long len) { const long o = (long)act_init.size(); act_init.resize(o + len, 1); return o; };
    for (auto &B : G) {
        auto pq = [&](int item) -> const pfmg_params & { return prob[B.probs[item / P]]; };
        B.o_dt_i = addd(B.items);
        B.o_nu_i = addd(B.items);
        B.o_dt_p = addd(B.nprob);
        B.o_nu_p = addd(B.nprob);
        for (int i = 0; i < B.items; ++i) {
            coef_host[B.o_dt_i + i] = pq(i).dt;
            coef_host[B.o_nu_i + i] = pq(i).nu;
        }
        for (int q = 0; q < B.nprob; ++q) {
            coef_host[B.o_dt_p + q] = prob[B.probs[q]].dt;
            coef_host[B.o_nu_p + q] = prob[B.probs[q]].nu;
        }
        for (int lev = 0; lev < nl; ++lev) {
            B.o_nu_f[lev] = addd((long)B.items * nn[lev]);
            for (long f = 0; f < (long)B.items * nn[lev]; ++f) coef_host[B.o_nu_f[lev] + f] = pq((int)(f / nn[lev])).nu;
            for (int m = 1; m < nn[lev]; ++m) {
                B.o_alpha_i[lev][m] = addd(B.items);
                B.o_delta_i[lev][m] = addd(B.items);
                B.o_alpha_p[lev][m] = addd(B.nprob);
                B.o_delta_p[lev][m] = addd(B.nprob);
                for (int i = 0; i < B.items; ++i) {
                    const double delta = pq(i).dt * d[lev][m];
                    coef_host[B.o_delta_i[lev][m] + i] = delta;
                    coef_host[B.o_alpha_i[lev][m] + i] = pq(i).nu * delta;
                }
                for (int q = 0; q < B.nprob; ++q) {
                    const pfmg_params &pr = prob[B.probs[q]];
                    const double delta = pr.dt * d[lev][m];
                    coef_host[B.o_delta_p[lev][m] + q] = delta;
                    coef_host[B.o_alpha_p[lev][m] + q] = pr.nu * delta;
                }
            }
        }
        B.o_from = addf((long)P * B.items);
        B.o_shift = addf((long)P * B.items);
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < B.items; ++i) {
                fixed_host[B.o_from + (long)j * B.items + i] = (i % P) >= j;
                fixed_host[B.o_shift + (long)j * B.items + i] = ((i + 1) % P) >= std::max(j, 1);
            }
        B.o_act_i = adda(B.items);
        B.o_act_p = adda(B.nprob);
        for (int lev = 0; lev < nl; ++lev) B.o_act_f[lev] = adda((long)B.items * nn[lev]);
        B.o_act_shift = adda(B.items);
        for (int i = 0; i < B.items; ++i) act_init[B.o_act_shift + i] = ((i + 1) % P) != 0;
    }
    active.assign(np, 1);
    res.assign(np, INFINITY);
    iters.assign(np, 0);
    return true;
}

// Lay out the workspace; with base == nullptr only the size is computed.
size_t BatchSolver::carve(char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~(size_t)255;
        char *r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    const bool mixed = p.precision == PFMG_MIXED;
    const bool jac = p.smoother == PFMG_SMOOTH_JACOBI;
    auto f64 = [&](int n, long count) -> double * {
        char *c = take((size_t)count * field_stride(n, dim, 8) * 8);
        return c ? (double *)c + field_lead(8) : nullptr;
    };
    auto f32 = [&](int n, long count) -> float * {
        char *c = take((size_t)count * field_stride(n, dim, 4) * 4);
        return c ? (float *)c + field_lead(4) : nullptr;
    };
    long dense_max = 0;
    for (auto &B : G) {
        dense_max = std::max(dense_max, interior_points(B.n, dim));
        for (int lev = 0; lev < nl; ++lev) {
            const int n = lev == 0 ? B.n : coarser(B.n);
            const int nnl = nn[lev];
            PLevel &L = B.L[lev];
            L.n = n;
            L.nn = nnl;
            L.fs = field_stride(n, dim, 8);
            L.U = f64(n, (long)B.items * nnl);
            L.F = f64(n, (long)B.items * nnl);
            L.I = f64(n, (long)B.items * (nnl - 1));
            L.B = f64(n, B.items);
            if (lev == 1) {
                L.Tau = f64(n, (long)B.items * nnl);
                L.Uold = f64(n, (long)B.items * nnl);
                L.DC = f64(n, (long)B.items * nn[0]);
            }
            L.mg.clear();
            for (int l = 0, m = n;; ++l, m = coarser(m)) {
                MGLevel M;
                M.n = m;
                M.fs64 = field_stride(m, dim, 8);
                M.fs32 = field_stride(m, dim, 4);
                if (l > 0) {
                    M.e = {f64(m, B.items), M.fs64};
                    M.b = {f64(m, B.items), M.fs64};
                }
                const bool pingpong = jac || (dim == 3 && m >= 31);
                if (pingpong) M.t = {f64(m, B.items), M.fs64};
                if (mixed) {
                    M.e32 = {f32(m, B.items), M.fs32};
                    M.b32 = {f32(m, B.items), M.fs32};
                    if (pingpong) M.t32 = {f32(m, B.items), M.fs32};
                }
                L.mg.push_back(M);
                if (m <= 2) break;
            }
        }
        B.ublock = f64(B.n, B.nprob);
        if (nl > 1) {
            B.ublock_c = f64(coarser(B.n), B.nprob);
            B.fublock_c = f64(coarser(B.n), B.nprob);
        }
    }
    for (int lev = 0; lev < nl; ++lev) {
        dQ[lev] = (double *)take(256 * 8);
        dS[lev] = (double *)take(256 * 8);
    }
    dLt = (double *)take(256 * 8);
    stage = (double *)take((size_t)dense_max * 8);
    bits = (unsigned long long *)take((size_t)2 * total_items * k::RSLOTS * 8);
    coef = (double *)take(coef_host.size() * 8);
    fixed_mask = (int *)take(fixed_host.size() * 4);
    act = (int *)take(act_init.size() * 4);
    return ((off + 255) & ~(size_t)255) + 256;
}

hipError_t BatchSolver::upload()
{
    static thread_local double Lt[256];
    for (int lev = 0; lev < nl; ++lev) {
        HC(hipMemcpyAsync(dQ[lev], Q[lev], sizeof(double) * nn[lev] * nn[lev], hipMemcpyHostToDevice, s));
        HC(hipMemcpyAsync(dS[lev], S[lev], sizeof(double) * nn[lev] * nn[lev], hipMemcpyHostToDevice, s));
    }
    if (nl > 1) {
        lagrange_interp(nn[0], s_ld[0], nn[1], s_ld[1], Lt);
        HC(hipMemcpyAsync(dLt, Lt, sizeof(double) * nn[0] * nn[1], hipMemcpyHostToDevice, s));
    }
    HC(hipMemcpyAsync(coef, coef_host.data(), coef_host.size() * 8, hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(fixed_mask, fixed_host.data(), fixed_host.size() * 4, hipMemcpyHostToDevice, s));
    std::memcpy(hact, act_init.data(), act_init.size() * 4);
    HC(hipMemcpyAsync(act, hact, act_init.size() * 4, hipMemcpyHostToDevice, s));
    act_dirty = false;
    return hipStreamSynchronize(s);
}

// ------------------------------------------------------------- multigrid
template <typename T, class Fn>
hipError_t BatchSolver::chunks(const std::vector<Leg<T>> &v, Fn fn) const
{
    for (size_t a = 0; a < v.size(); a += MAXSEG) {
        const int ns = (int)std::min<size_t>(MAXSEG, v.size() - a);
        const Leg<T> &h = v[a];
        Tiling t{h.n, dim, h.count, h.mask, noremap, h.alpha, ns};
        for (int w = 1; w < ns; ++w) {
            const Leg<T> &x = v[a + w];
            t.x[w - 1] = SegX{x.n, x.count, x.mask, x.alpha};
        }
        HC(fn(t, &v[a], ns));
    }
    return hipSuccess;
}

template <typename T>
hipError_t BatchSolver::smooth(const std::vector<Leg<T>> &legs, int sweeps, bool from_zero)
{
    const double om = p.omega;
    return chunks(legs, [&](const Tiling &t, const Leg<T> *x, int ns) -> hipError_t {
        View<T> u = cat(x, ns, [](const Leg<T> &l) { return l.u; });
        View<T> b = cat(x, ns, [](const Leg<T> &l) { return l.b; });
        View<T> tmp = cat(x, ns, [](const Leg<T> &l) { return l.t; });
        if (sweeps == 0) return from_zero ? k::zero(t, u, s) : hipSuccess;
        bool fusable = p.smoother == PFMG_SMOOTH_RBGS && dim == 3;
        long pts = 0;
        for (int w = 0; w < ns; ++w) {
            fusable = fusable && x[w].n >= 31 && x[w].n <= 255 && x[w].t.p;
            pts += (long)x[w].count * interior_points(x[w].n, dim);
        }
        RbPlan plan;
        if (fusable) plan = rb_plan<T>(t, 0.0, om, b, u, tmp, s, pts >= fused_min_points);
        if (plan.fused) {
            // timing family "rbgs@<largest n of the launch>"
            int nmax = 0;
            for (int w = 0; w < ns; ++w) nmax = std::max(nmax, x[w].n);
            View<T> src = u, dst = tmp;
            for (int q = 0; q < sweeps; ++q) {
                timer.start("rbgs", nmax, 3.0 * sizeof(T), pts, true, s);
                const hipError_t e = k::rbgs_fused(t, 0.0, om, q == 0 && from_zero, b, src, dst, s, &plan.shape);
                timer.stop(s);
                HC(e);
                std::swap(src, dst);
            }
            if (src.p != u.p) HC(k::copy(t, src, u, s));
            return hipSuccess;
        }
        if (p.smoother == PFMG_SMOOTH_RBGS) {
            for (int q = 0; q < sweeps; ++q) {
                if (q == 0 && from_zero) HC(k::rbgs_zero_red(t, 0.0, om, b, u, s));
                else HC(k::rbgs(t, 0.0, om, 0, b, u, s));
                HC(k::rbgs(t, 0.0, om, 1, b, u, s));
            }
            return hipSuccess;
        }
        View<T> src = u, dst = tmp;
        for (int q = 0; q < sweeps; ++q) {
            if (q == 0 && from_zero) HC(k::jacobi_zero(t, 0.0, om, b, dst, s));
            else HC(k::jacobi(t, 0.0, om, b, src, dst, s));
            std::swap(src, dst);
        }
        if (src.p != u.p) HC(k::copy(t, src, u, s));
        return hipSuccess;
    });
}

// One V(nu_pre, nu_post)-cycle for every leg (depth 0 of its group's
// hierarchy); zero_top starts from u = 0 (the correction of a refinement
// step) instead of the leg's u.
template <typename T>
hipError_t BatchSolver::vcycle(std::vector<Leg<T>> legs, bool zero_top)
{
    std::vector<std::vector<Leg<T>>> down;
    std::vector<Leg<T>> bottom[2], exact;
    for (int dd = 0; !legs.empty(); ++dd) {
        std::vector<Leg<T>> go, next;
        for (const Leg<T> &x : legs) {
            const bool zero = dd > 0 || zero_top;
            if (use_bottom && k::vcycle_bottom_lds(x.n, dim, p.smoother, sizeof(T)) <= k::bottom_lds_max()) {
                bottom[zero ? 1 : 0].push_back(x);
            } else if (x.n <= 2) {
                exact.push_back(x);
            } else {
                go.push_back(x);
                const MGLevel &M = G[x.g].L[x.lev].mg[dd + 1];
                Leg<T> y = x;
                y.d = dd + 1;
                y.n = M.n;
                y.u = mg_e<T>(M);
                y.b = mg_b<T>(M);
                y.t = mg_t<T>(M);
                next.push_back(y);
            }
        }
        down.push_back(go);
        legs.swap(next);
    }
    for (size_t dd = 0; dd < down.size(); ++dd) {
        if (down[dd].empty()) continue;
        HC(smooth<T>(down[dd], p.nu_pre, dd > 0 || zero_top));
        HC(chunks(down[dd], [&](const Tiling &t, const Leg<T> *x, int ns) {
            View<T> bc = cat(x, ns, [&](const Leg<T> &l) { return mg_b<T>(G[l.g].L[l.lev].mg[l.d + 1]); });
            return k::resid_restrict(t, 0.0, cat(x, ns, [](const Leg<T> &l) { return l.b; }),
                                     cat(x, ns, [](const Leg<T> &l) { return l.u; }), bc, s);
        }));
    }
    for (int z = 0; z < 2; ++z)
        HC(chunks(bottom[z], [&](const Tiling &t, const Leg<T> *x, int ns) {
            return k::vcycle_bottom(t, 0.0, p.smoother, p.omega, p.nu_pre, p.nu_post, z == 1,
                                    cat(x, ns, [](const Leg<T> &l) { return l.b; }),
                                    cat(x, ns, [](const Leg<T> &l) { return l.u; }), s);
        }));
    HC(chunks(exact, [&](const Tiling &t, const Leg<T> *x, int ns) {
        return k::coarsest(t, 0.0, cat(x, ns, [](const Leg<T> &l) { return l.b; }),
                           cat(x, ns, [](const Leg<T> &l) { return l.u; }), s);
    }));
    for (size_t q = down.size(); q-- > 0;) {
        if (down[q].empty()) continue;
        HC(chunks(down[q], [&](const Tiling &t, const Leg<T> *x, int ns) {
            View<T> ec = cat(x, ns, [&](const Leg<T> &l) { return mg_e<T>(G[l.g].L[l.lev].mg[l.d + 1]); });
            return k::prolong_add(t, ec, cat(x, ns, [](const Leg<T> &l) { return l.u; }), s);
        }));
        HC(smooth<T>(down[q], p.nu_post, false));
    }
    return hipSuccess;
}

// One V-cycle, or one refinement step of the mixed form: FP64 residual
// rounded to FP32, FP32 V-cycle from a zero correction, FP64 update.
hipError_t BatchSolver::cycle_step(const std::vector<Leg<double>> &top)
{
    if (p.precision != PFMG_MIXED) return vcycle<double>(top, false);
    std::vector<Leg<float>> low;
    for (const Leg<double> &x : top) {
        const MGLevel &M = G[x.g].L[x.lev].mg[0];
        low.push_back(Leg<float>{x.g, x.lev, 0, x.n, x.count, x.mask, x.alpha, M.e32, M.b32, M.t32});
    }
    HC(chunks(top, [&](const Tiling &t, const Leg<double> *x, int ns) {
        View<float> b32 = cat(low.data() + (x - top.data()), ns, [](const Leg<float> &l) { return l.b; });
        return k::resid_round(t, 0.0, cat(x, ns, [](const Leg<double> &l) { return l.b; }),
                              cat(x, ns, [](const Leg<double> &l) { return l.u; }), b32, s);
    }));
    HC(vcycle<float>(low, true));
    return chunks(top, [&](const Tiling &t, const Leg<double> *x, int ns) {
        View<float> e32 = cat(low.data() + (x - top.data()), ns, [](const Leg<float> &l) { return l.u; });
        return k::add_f32(t, e32, cat(x, ns, [](const Leg<double> &l) { return l.u; }), s);
    });
}

// ------------------------------------------------------------------- SDC
// One sweep (eq. sdc-be with the node solves of Sec. 2.3.1) on level lev.
// chain >= 0: slice `chain` of every problem (a step of the coarse chain);
// chain < 0: every item, masked by predictor round `round` when
// masked_round, else by the active mask.
hipError_t BatchSolver::sweep(int lev, int chain, bool masked_round, int round)
{
    const int nnl = nn[lev];
    const bool ch = chain >= 0;
    const long p0 = ch ? chain : 0, mul = ch ? P : 1;
    auto count = [&](const BGroup &B) { return ch ? B.nprob : B.items; };
    auto mask = [&](const BGroup &B) -> const int * {
        if (ch) return AM(B.o_act_p);
        if (masked_round) return round > 0 ? FM(B.o_from + (long)round * B.items) : nullptr;
        return AM(B.o_act_i);
    };
    std::vector<Seg> r(ng);
    for (int g = 0; g < ng; ++g) {
        const BGroup &B = G[g];
        const PLevel &L = B.L[lev];
        const long sst = (long)nnl * L.fs, ist = (long)(nnl - 1) * L.fs;
        r[g] = Seg{L.n, count(B), mask(B), C(ch ? B.o_dt_p : B.o_dt_i), {}};
        r[g].v[0] = {L.slot(L.F, (int)p0, 0), mul * sst};
        r[g].v[1] = {L.I + p0 * ist, mul * ist};
    }
    HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
        return k::sdc_integrals(t, nnl, 0.0, dS[lev], v[0], v[1], s);
    }));
    for (int m = 0; m + 1 < nnl; ++m) {
        std::vector<Leg<double>> legs;
        for (int g = 0; g < ng; ++g) {
            const BGroup &B = G[g];
            const PLevel &L = B.L[lev];
            const long sst = (long)nnl * L.fs, ist = (long)(nnl - 1) * L.fs;
            Seg &x = r[g];
            x.coef = C(ch ? B.o_delta_p[lev][m + 1] : B.o_delta_i[lev][m + 1]);
            x.v[0] = {L.slot(L.U, (int)p0, m), mul * sst};
            x.v[1] = {L.slot(L.F, (int)p0, m + 1), mul * sst};
            x.v[2] = {L.I + p0 * ist + (long)m * L.fs, mul * ist};
            x.v[3] = lev == 1 ? View<double>{L.slot(L.Tau, (int)p0, m + 1), mul * sst} : View<double>{nullptr, 0};
            x.v[4] = lev == 1 ? View<double>{L.slot(L.Tau, (int)p0, m), mul * sst} : View<double>{nullptr, 0};
            x.v[5] = {L.B, L.fs};
            legs.push_back(Leg<double>{g, lev, 0, L.n, x.count, x.mask,
                                       C(ch ? B.o_alpha_p[lev][m + 1] : B.o_alpha_i[lev][m + 1]),
                                       View<double>{L.slot(L.U, (int)p0, m + 1), mul * sst}, View<double>{L.B, L.fs},
                                       L.mg[0].t});
        }
        HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
            return k::sdc_rhs(t, 0.0, v[0], v[1], v[2], v[3], v[4], v[5], s);
        }));
        for (int c = 0; c < p.vcycles_per_solve; ++c) HC(cycle_step(legs));
        std::vector<Seg> fl(ng);
        for (int g = 0; g < ng; ++g) {
            const BGroup &B = G[g];
            fl[g] = Seg{legs[g].n, legs[g].count, legs[g].mask, C(ch ? B.o_nu_p : B.o_nu_i), {}};
            fl[g].v[0] = legs[g].u;
            fl[g].v[1] = r[g].v[1];
        }
        HC(for_segs(fl, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
            return k::apply_L(t, 0.0, v[0], v[1], s);
        }));
    }
    return hipSuccess;
}

// FAS restriction (Sec. 2.3) of every item; masked: active problems only.
hipError_t BatchSolver::fas_restrict(bool masked)
{
    std::vector<Seg> a(ng), b(ng);
    for (int g = 0; g < ng; ++g) {
        const BGroup &B = G[g];
        const PLevel &Fn = B.L[0], &Cs = B.L[1];
        const long fst = (long)Fn.nn * Fn.fs, cst = (long)Cs.nn * Cs.fs;
        a[g] = Seg{Cs.n, B.items, masked ? AM(B.o_act_i) : nullptr, C(B.o_dt_i), {}};
        a[g].v[0] = {Fn.U, fst};
        a[g].v[1] = {Fn.F, fst};
        a[g].v[2] = {Cs.U, cst};
        a[g].v[3] = {Cs.Uold, cst};
        a[g].v[4] = {Cs.Tau, cst};
        a[g].v[5] = {Cs.F, cst};
        b[g] = Seg{Cs.n, B.items * Cs.nn, masked ? AM(B.o_act_f[1]) : nullptr, C(B.o_nu_f[1]), {}};
        b[g].v[0] = {Cs.U, Cs.fs};
        b[g].v[1] = {Cs.F, Cs.fs};
    }
    HC(for_segs(a, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
        return k::fas_inject(t, nn[0], nn[1], cmap, 0.0, dQ[0], v[0], v[1], v[2], v[3], v[4], s);
    }));
    HC(for_segs(b, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
        return k::apply_L(t, 0.0, v[0], v[1], s);
    }));
    return for_segs(a, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
        return k::fas_tau(t, nn[1], 0.0, dQ[1], v[5], v[4], s);
    });
}

// Interpolation of the coarse corrections to all fine nodes, then F.
hipError_t BatchSolver::interpolate(bool masked)
{
    std::vector<Seg> a(ng), b(ng);
    for (int g = 0; g < ng; ++g) {
        const BGroup &B = G[g];
        const PLevel &Fn = B.L[0], &Cs = B.L[1];
        const long cst = (long)Cs.nn * Cs.fs;
        a[g] = Seg{Cs.n, B.items, masked ? AM(B.o_act_i) : nullptr, nullptr, {}};
        a[g].v[0] = {Cs.U, cst};
        a[g].v[1] = {Cs.Uold, cst};
        a[g].v[2] = {Cs.DC, (long)Fn.nn * Cs.fs};
        b[g] = Seg{Fn.n, B.items * Fn.nn, masked ? AM(B.o_act_f[0]) : nullptr, C(B.o_nu_f[0]), {}};
        b[g].v[0] = {Cs.DC, Cs.fs};
        b[g].v[1] = {Fn.U, Fn.fs};
        b[g].v[2] = {Fn.F, Fn.fs};
    }
    HC(for_segs(a, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
        return k::interp_coarse(t, nn[0], nn[1], dLt, v[0], v[1], v[2], s);
    }));
    HC(for_segs(b, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
        return k::prolong_add(t, v[0], v[1], s);
    }));
    return for_segs(b, dim, noremap, [&](const Tiling &t, View<double> *v, int) {
        return k::apply_L(t, 0.0, v[1], v[2], s);
    });
}

// Block start after every u_block is in place: spread to all nodes and
// slices, F, the injected coarse initial values and the predictor
// (Sec. 2.4: round j sweeps the coarse slices p >= j of every problem,
// after slice p takes slice p-1's end value of round j-1).
hipError_t BatchSolver::spread_body()
{
    for (int pp = 0; pp < P; ++pp)
        for (int m = 0; m < nn[0]; ++m) {
            std::vector<Seg> r(ng);
            for (int g = 0; g < ng; ++g) {
                const BGroup &B = G[g];
                const PLevel &Fn = B.L[0];
                r[g] = Seg{Fn.n, B.nprob, nullptr, nullptr, {}};
                r[g].v[0] = {B.ublock, Fn.fs};
                r[g].v[1] = {Fn.slot(Fn.U, pp, m), (long)P * Fn.nn * Fn.fs};
            }
            HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::copy(t, v[0], v[1], s); }));
        }
    {
        std::vector<Seg> r(ng);
        for (int g = 0; g < ng; ++g) {
            const BGroup &B = G[g];
            const PLevel &Fn = B.L[0];
            r[g] = Seg{Fn.n, B.items * Fn.nn, nullptr, C(B.o_nu_f[0]), {}};
            r[g].v[0] = {Fn.U, Fn.fs};
            r[g].v[1] = {Fn.F, Fn.fs};
        }
        HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::apply_L(t, 0.0, v[0], v[1], s); }));
    }
    if (nl < 2) return hipSuccess;
    {
        std::vector<Seg> r(ng);
        for (int g = 0; g < ng; ++g) {
            const BGroup &B = G[g];
            const PLevel &Fn = B.L[0], &Cs = B.L[1];
            r[g] = Seg{Cs.n, B.nprob, nullptr, C(B.o_nu_p), {}};
            r[g].v[0] = {B.ublock, Fn.fs};
            r[g].v[1] = {B.ublock_c, Cs.fs};
            r[g].v[2] = {B.fublock_c, Cs.fs};
        }
        HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::inject(t, v[0], v[1], s); }));
        HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::apply_L(t, 0.0, v[1], v[2], s); }));
    }
    HC(fas_restrict(false));
    const int Mc = nn[1] - 1;
    for (int j = 0; j < P; ++j) {
        if (j >= 1) {
            std::vector<Seg> r(ng);
            for (int g = 0; g < ng; ++g) {
                const BGroup &B = G[g];
                const PLevel &Cs = B.L[1];
                const long cst = (long)Cs.nn * Cs.fs;
                r[g] = Seg{Cs.n, B.items - 1, FM(B.o_shift + (long)j * B.items), nullptr, {}};
                r[g].v[0] = {Cs.slot(Cs.U, 0, Mc), cst};
                r[g].v[1] = {Cs.slot(Cs.U, 1, 0), cst};
                r[g].v[2] = {Cs.slot(Cs.F, 0, Mc), cst};
                r[g].v[3] = {Cs.slot(Cs.F, 1, 0), cst};
            }
            HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::copy(t, v[0], v[1], s); }));
            HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::copy(t, v[2], v[3], s); }));
        }
        HC(sweep(1, -1, true, j));
    }
    return interpolate(false);
}

// One iteration of every active problem, ending with the residual partials.
hipError_t BatchSolver::iterate_body()
{
    const int M = nn[0] - 1;
    {
        std::vector<Seg> r(ng);
        for (int g = 0; g < ng; ++g) {
            const BGroup &B = G[g];
            const PLevel &Fn = B.L[0];
            const long fst = (long)Fn.nn * Fn.fs;
            r[g] = Seg{Fn.n, B.items - 1, AM(B.o_act_shift), nullptr, {}};
            r[g].v[0] = {Fn.slot(Fn.U, 0, M), fst};
            r[g].v[1] = {Fn.slot(Fn.U, 1, 0), fst};
            r[g].v[2] = {Fn.slot(Fn.F, 0, M), fst};
            r[g].v[3] = {Fn.slot(Fn.F, 1, 0), fst};
        }
        HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::copy(t, v[0], v[1], s); }));
        HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::copy(t, v[2], v[3], s); }));
    }
    HC(sweep(0, -1, false, 0));
    if (nl > 1) {
        HC(fas_restrict(true));
        const int Mc = nn[1] - 1;
        for (int pp = 0; pp < P; ++pp) {
            std::vector<Seg> r(ng);
            for (int g = 0; g < ng; ++g) {
                const BGroup &B = G[g];
                const PLevel &Cs = B.L[1];
                const long cst = (long)Cs.nn * Cs.fs;
                r[g] = Seg{Cs.n, B.nprob, AM(B.o_act_p), nullptr, {}};
                if (pp == 0) {
                    r[g].v[0] = {B.ublock_c, Cs.fs};
                    r[g].v[2] = {B.fublock_c, Cs.fs};
                } else {
                    r[g].v[0] = {Cs.slot(Cs.U, pp - 1, Mc), (long)P * cst};
                    r[g].v[2] = {Cs.slot(Cs.F, pp - 1, Mc), (long)P * cst};
                }
                r[g].v[1] = {Cs.slot(Cs.U, pp, 0), (long)P * cst};
                r[g].v[3] = {Cs.slot(Cs.F, pp, 0), (long)P * cst};
            }
            HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::copy(t, v[0], v[1], s); }));
            HC(for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int) { return k::copy(t, v[2], v[3], s); }));
            HC(sweep(1, pp, false, 0));
        }
        HC(interpolate(true));
    }
    // collocation residual (eq. resid): RSLOTS partial maxima per item
    HC(k::fill_u64(bits, 0, 2 * total_items * k::RSLOTS, s));
    std::vector<Seg> r(ng);
    for (int g = 0; g < ng; ++g) {
        const BGroup &B = G[g];
        const PLevel &Fn = B.L[0];
        const long fst = (long)Fn.nn * Fn.fs;
        r[g] = Seg{Fn.n, B.items, AM(B.o_act_i), C(B.o_dt_i), {}};
        r[g].v[0] = {Fn.U, fst};
        r[g].v[1] = {Fn.F, fst};
        r[g].v[2] = {B.ublock, Fn.fs};
    }
    return for_segs(r, dim, noremap, [&](const Tiling &t, View<double> *v, int first) {
        const long f0 = G[first].item0;
        return k::colloc_resid(t, nn[0], P, 0.0, dQ[0], v[0], v[1], v[2], bits + f0 * k::RSLOTS,
                               bits + ((long)total_items + f0) * k::RSLOTS, s);
    });
}

// --------------------------------------------------------------- driver
hipError_t BatchSolver::set_initial(const double *u0, bool on_device)
{
    long off = 0;
    for (int q = 0; q < NP; ++q) {
        const BGroup &B = G[grp_of[q]];
        const PLevel &Fn = B.L[0];
        const long pts = interior_points(B.n, dim);
        const double *src = u0 + off;
        if (!on_device) {
            HC(hipMemcpyAsync(stage, src, sizeof(double) * pts, hipMemcpyHostToDevice, s));
            src = stage;
        }
        HC(k::unpack(Tiling{B.n, dim, 1, nullptr, noremap}, src,
                     View<double>{B.ublock + (long)loc_of[q] * Fn.fs, 0}, s));
        off += pts;
    }
    active.assign(NP, 1);
    res.assign(NP, INFINITY);
    iters.assign(NP, 0);
    nan = false;
    if (use_graph() && warm_start) {
        if (!g_start) HC(capture([this] { return spread_body(); }, &g_start));
        HC(hipGraphLaunch(g_start, s));
    } else {
        warm_start = true;   // first block start eagerly: launch shapes are tuned outside capture
        HC(spread_body());
    }
    if (nl > 1) vcount[1] += (long long)NP * P * (P + 1) / 2 * (nn[1] - 1) * p.vcycles_per_solve;
    // every problem iterates again
    HC(hipStreamSynchronize(s));
    std::memcpy(hact, act_init.data(), act_init.size() * 4);
    act_dirty = true;
    has_state = true;
    return hipSuccess;
}

void BatchSolver::freeze(int q)
{
    BGroup &B = G[grp_of[q]];
    const int lq = loc_of[q];
    active[q] = 0;
    hact[B.o_act_p + lq] = 0;
    for (int pp = 0; pp < P; ++pp) {
        const int item = lq * P + pp;
        hact[B.o_act_i + item] = 0;
        for (int lev = 0; lev < nl; ++lev)
            for (int m = 0; m < nn[lev]; ++m) hact[B.o_act_f[lev] + (long)item * nn[lev] + m] = 0;
        if (pp >= 1) hact[B.o_act_shift + item - 1] = 0;
    }
    act_dirty = true;
}

hipError_t BatchSolver::iterate()
{
    if (act_dirty) {
        HC(hipMemcpyAsync(act, hact, act_init.size() * 4, hipMemcpyHostToDevice, s));
        act_dirty = false;
    }
    long act_items = 0;
    for (int q = 0; q < NP; ++q) act_items += active[q] ? P : 0;
    if (use_graph() && warm_iter) {
        if (!g_iter) HC(capture([this] { return iterate_body(); }, &g_iter));
        HC(hipGraphLaunch(g_iter, s));
    } else {
        warm_iter = true;
        HC(iterate_body());
    }
    vcount[0] += act_items * (nn[0] - 1) * p.vcycles_per_solve;
    if (nl > 1) vcount[1] += act_items * (nn[1] - 1) * p.vcycles_per_solve;
    const long nb = 2L * total_items * k::RSLOTS;
    HC(hipMemcpyAsync(hbits, bits, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    for (int q = 0; q < NP; ++q) {
        if (!active[q]) continue;
        const BGroup &B = G[grp_of[q]];
        double worst = 0;
        for (int pp = 0; pp < P; ++pp) {
            const long item = B.item0 + (long)loc_of[q] * P + pp;
            unsigned long long rb = 0, ub = 0;
            for (int w = 0; w < k::RSLOTS; ++w) {
                rb = std::max(rb, hbits[item * k::RSLOTS + w]);
                ub = std::max(ub, hbits[((long)total_items + item) * k::RSLOTS + w]);
            }
            const double r = bits_to_double(rb), u0 = bits_to_double(ub);
            const double v = u0 > 0 ? r / u0 : r;
            if (!std::isfinite(v)) nan = true;
            if (v > worst || v != v) worst = v;
        }
        res[q] = worst;
        iters[q] += 1;
        if (worst <= p.pfasst_tol) freeze(q);
    }
    return hipSuccess;
}

hipError_t BatchSolver::get(int q, int field, int slice, int node, double *dst, bool on_device)
{
    const BGroup &B = G[grp_of[q]];
    const bool coarse = field >= PFMG_U_COARSE;
    const PLevel &Lv = B.L[coarse ? 1 : 0];
    double *base = nullptr;
    switch (field) {
    case PFMG_U_FINE: case PFMG_U_COARSE: base = Lv.U; break;
    case PFMG_F_FINE: case PFMG_F_COARSE: base = Lv.F; break;
    case PFMG_TAU: base = Lv.Tau; break;
    default: base = Lv.Uold; break;
    }
    double *f = Lv.slot(base, loc_of[q] * P + slice, node);
    double *target = on_device ? dst : stage;
    HC(k::pack(Tiling{Lv.n, dim, 1, nullptr, noremap}, View<double>{f, 0}, target, s));
    if (!on_device)
        HC(hipMemcpyAsync(dst, stage, sizeof(double) * interior_points(Lv.n, dim), hipMemcpyDeviceToHost, s));
    return hipStreamSynchronize(s);
}

hipError_t BatchSolver::capture(const std::function<hipError_t()> &fn, hipGraphExec_t *out)
{
    if (!cap) HC(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t saved = s;
    s = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    hipError_t e1 = e == hipSuccess ? fn() : e;
    hipGraph_t g = nullptr;
    hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cap, &g) : e;
    s = saved;
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e1 != hipSuccess ? e1 : e2;
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

void BatchSolver::release()
{
    if (g_iter) (void)hipGraphExecDestroy(g_iter);
    if (g_start) (void)hipGraphExecDestroy(g_start);
    if (cap) (void)hipStreamDestroy(cap);
    g_iter = g_start = nullptr;
    cap = nullptr;
}

template hipError_t BatchSolver::vcycle<double>(std::vector<Leg<double>>, bool);
template hipError_t BatchSolver::vcycle<float>(std::vector<Leg<float>>, bool);

}  // namespace pfmg
