// IPFASST on one GPU: the P time slices of a block are processed together;
// each "time rank" of the paper is a slice of the batched state.
//
// Per iteration (Sec. 2.4): new fine initial values from the previous
// slices (their end values after the previous iteration), one fine SDC
// sweep on all slices at once, FAS restriction, the coarse sweeps in slice
// order (the blocking coarse level of PFASST), interpolation of the coarse
// correction, and the collocation residual (eq. resid).  Every node solve
// is a fixed number of V-cycles (IMLSDC, Sec. 2.3.1) or a full solve
// (Sec. 4.2.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "collocation.h"
#include "solver.h"
#include "tune.h"
#include "unet.h"

#define HC(x)                                  \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

namespace pfmg {

static inline double bits_to_double(unsigned long long b)
{
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

bool Solver::validate(const pfmg_params &p, std::string &why)
{
    if (p.dim != 1 && p.dim != 3) { why = "dim must be 1 or 3"; return false; }
    if (p.n < 1) { why = "n must be >= 1"; return false; }
    for (int n = p.n; n > 2; n = coarser(n))
        if ((n & 1) == 0) { why = "every multigrid level with n >= 3 must be odd"; return false; }
    if (!(p.nu > 0) || !(p.dt > 0) || !std::isfinite(p.nu) || !std::isfinite(p.dt)) {
        why = "nu and dt must be positive and finite"; return false;
    }
    if (p.n_slices < 1 || p.n_slices > 4096) { why = "n_slices must be in 1..4096"; return false; }
    if (p.nodes_fine < 2 || p.nodes_fine > 9) { why = "nodes_fine must be in 2..9"; return false; }
    if (p.node_family != PFMG_NODES_LOBATTO && p.node_family != PFMG_NODES_UNIFORM) {
        why = "node_family must be PFMG_NODES_LOBATTO or PFMG_NODES_UNIFORM"; return false;
    }
    if (p.nodes_middle != 0 && (p.nodes_coarse == 0 || p.nodes_middle < 2 || p.nodes_middle > p.nodes_fine)) {
        why = "nodes_middle needs a coarse level and must be in 2..nodes_fine"; return false;
    }
    if (p.nodes_coarse != 0) {
        const int nlv = levels(p);
        if (p.nodes_coarse < 2 || p.nodes_coarse > level_nodes(p, nlv - 2)) { why = "bad nodes_coarse"; return false; }
        if (p.n < 3 || (nlv == 3 && coarser(p.n) < 3)) { why = "every coarser level needs n >= 3 above it"; return false; }
        for (int l = 1; l < nlv; ++l) {
            long double sf[16], sc[16];
            const int nf = level_nodes(p, l - 1), nc = level_nodes(p, l);
            if (!family_nodes_ld(p.node_family, nf, sf) || !family_nodes_ld(p.node_family, nc, sc)) {
                why = "node construction failed"; return false;
            }
            for (int mc = 0; mc < nc; ++mc) {
                bool found = false;
                for (int mf = 0; mf < nf; ++mf) found = found || std::fabs((double)(sf[mf] - sc[mc])) < 1e-14;
                if (!found) { why = "a level's nodes must be a subset of the finer level's (injection in time)"; return false; }
            }
        }
    }
    if (p.smoother != PFMG_SMOOTH_JACOBI && p.smoother != PFMG_SMOOTH_RBGS) { why = "bad smoother"; return false; }
    if (p.stencil_order != 2 && p.stencil_order != 4) { why = "stencil_order must be 2 or 4"; return false; }
    if (p.interp_order != 2 && p.interp_order != 4) { why = "interp_order must be 2 or 4"; return false; }
    if ((p.f_solve != 0 && p.f_solve != 1) || (p.f_interp != 0 && p.f_interp != 1)) {
        why = "f_solve and f_interp must be 0 or 1"; return false;
    }
    if (p.residual_abs != 0 && p.residual_abs != 1) { why = "residual_abs must be 0 or 1"; return false; }
    if (p.stencil_order == 4 && (p.precision != PFMG_FP64 || p.guess != PFMG_GUESS_PREV)) {
        why = "stencil_order 4 needs FP64 and plain guesses"; return false;
    }
    if (p.stencil_order == 4 && p.n < 3) { why = "stencil_order 4 needs n >= 3"; return false; }
    if (p.interp_order == 4 && p.nodes_coarse > 0 &&
        coarser(levels(p) == 3 ? coarser(p.n) : p.n) < 3) {
        why = "cubic interpolation needs a coarse grid of n >= 3"; return false;
    }
    if (p.nu_pre < 0 || p.nu_post < 0 || p.nu_pre + p.nu_post == 0 || p.nu_pre > 16 || p.nu_post > 16) {
        why = "smoothing sweeps must be in 0..16 and not both 0"; return false;
    }
    if (!(p.omega > 0 && p.omega < 2)) { why = "omega must be in (0, 2)"; return false; }
    if (p.vcycles_per_solve < 0 || p.vcycles_per_solve > 100) { why = "vcycles_per_solve in 0..100"; return false; }
    if (p.vcycles_per_solve == 0 && (p.mg_max_cycles < 1 || !(p.mg_tol >= 0) || !(p.mg_stall > 0))) {
        why = "full solves need mg_max_cycles >= 1, mg_tol >= 0, mg_stall > 0"; return false;
    }
    if (p.precision != PFMG_FP64 && p.precision != PFMG_MIXED) { why = "bad precision"; return false; }
    if (p.guess != PFMG_GUESS_PREV && p.guess != PFMG_GUESS_LEARNED) { why = "bad guess"; return false; }
    if (p.guess == PFMG_GUESS_LEARNED && (p.dim != 3 || p.vcycles_per_solve != 0 || !UNet::valid_n(p.n) ||
                                          (p.smoother == PFMG_SMOOTH_RBGS && p.n < 31))) {
        why = "the learned guess needs 3D full solves (vcycles_per_solve = 0) and a network grid: n odd over three "
              "levels, n >= 31 with red-black smoothing";
        return false;
    }
    if (p.fine_send != PFMG_SEND_AFTER_ITER && p.fine_send != PFMG_SEND_AFTER_SWEEP) {
        why = "fine_send must be PFMG_SEND_AFTER_ITER or PFMG_SEND_AFTER_SWEEP"; return false;
    }
    if (p.pfasst_max_iter < 1) { why = "pfasst_max_iter must be >= 1"; return false; }
    if (!(p.guess_min_relres >= 0)) { why = "guess_min_relres must be >= 0"; return false; }
    return true;
}

// Lay out the workspace.  With base == nullptr only the size is computed.
size_t Solver::carve(const pfmg_params &p, char *base, Solver *sv)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~(size_t)255;
        char *r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    const int dim = p.dim, P = p.n_slices;
    const int nl = levels(p);
    const bool mixed = p.precision == PFMG_MIXED;
    const bool jac = p.smoother == PFMG_SMOOTH_JACOBI;
    auto f64 = [&](int n, long count) -> double * {
        const long fs = field_stride(n, dim, 8);
        char *c = take((size_t)count * fs * 8);
        return c ? (double *)c + field_lead(8) : nullptr;
    };
    auto f32 = [&](int n, long count) -> float * {
        const long fs = field_stride(n, dim, 4);
        char *c = take((size_t)count * fs * 4);
        return c ? (float *)c + field_lead(4) : nullptr;
    };
    for (int lev = 0, n = p.n; lev < nl; ++lev, n = coarser(n)) {
        const int nn = level_nodes(p, lev);
        PLevel tmp;
        PLevel &L = sv ? sv->L[lev] : tmp;
        L.n = n;
        L.nn = nn;
        L.fs = field_stride(n, dim, 8);
        L.U = f64(n, (long)P * nn);
        L.F = f64(n, (long)P * nn);
        L.I = f64(n, (long)P * (nn - 1));
        L.B = f64(n, P);
        if (lev >= 1) {
            L.Tau = f64(n, (long)P * nn);
            L.Uold = f64(n, (long)P * nn);
            L.DC = f64(n, (long)P * level_nodes(p, lev - 1));
            L.DCF = p.f_interp ? f64(n, (long)P * level_nodes(p, lev - 1)) : nullptr;
            L.Fold = p.f_interp ? f64(n, (long)P * nn) : nullptr;
        }
        // F(U) of every fine node for the collocation residual when the
        // stored F is not F(U)
        L.Ft = lev == 0 && (p.f_solve || p.f_interp) ? f64(n, (long)P * nn) : nullptr;
        L.mg.clear();
        for (int l = 0, nl_ = n;; ++l, nl_ = coarser(nl_)) {
            MGLevel G;
            G.n = nl_;
            G.fs64 = field_stride(nl_, dim, 8);
            G.fs32 = field_stride(nl_, dim, 4);
            if (l > 0) {
                G.e = {f64(nl_, P), G.fs64};
                G.b = {f64(nl_, P), G.fs64};
            }
            // second buffer for out-of-place sweeps (Jacobi, fused red-black,
            // the fourth-order smoother and residual on the fine level's
            // finest grid)
            const bool pingpong = jac || (dim == 3 && nl_ >= 31) || (lev == 0 && l == 0 && p.stencil_order == 4);
            if (pingpong) G.t = {f64(nl_, P), G.fs64};
            if (mixed) {
                G.e32 = {f32(nl_, P), G.fs32};
                G.b32 = {f32(nl_, P), G.fs32};
                if (pingpong) G.t32 = {f32(nl_, P), G.fs32};
            }
            L.mg.push_back(G);
            if (nl_ <= 2) break;
        }
        double *dQ = (double *)take(256 * 8), *dS = (double *)take(256 * 8);
        L.dQ = dQ;
        L.dS = dS;
    }
    double *ub = f64(p.n, 1), *vb = f64(p.n, 1), *vu = f64(p.n, 1);
    // the fine end values kept right after the fine sweeps (AFTER_SWEEP)
    double *esnap = p.fine_send == PFMG_SEND_AFTER_SWEEP ? f64(p.n, P) : nullptr;
    double *ubc = nullptr, *fubc = nullptr, *ubm = nullptr;
    if (nl > 1) {
        const int nc = nl == 3 ? coarser(coarser(p.n)) : coarser(p.n);
        ubc = f64(nc, 1);
        fubc = f64(nc, 1);
        if (nl == 3) ubm = f64(coarser(p.n), 1);
    }
    double *lt = (double *)take(256 * 8), *lt2 = (double *)take(256 * 8);
    auto *bits = (unsigned long long *)take((size_t)4 * P * k::RSLOTS * 8);
    int *mask = (int *)take((size_t)P * 4);
    double *nnsc = (double *)take((size_t)2 * P * 8);
    if (sv) {
        sv->ublock = ub;
        sv->esnap = esnap;
        sv->vb = vb;
        sv->vu = vu;
        sv->ublock_c = ubc;
        sv->fublock_c = fubc;
        sv->ublock_m = ubm;
        sv->dLt[0] = lt;
        sv->dLt[1] = lt2;
        sv->bits = bits;
        sv->mask = mask;
        sv->nnsc = nnsc;
    }
    return ((off + 255) & ~(size_t)255) + 256;
}

size_t Solver::carve_vcycle(const pfmg_params &p, char *base, Solver *sv)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~(size_t)255;
        char *r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    const int dim = p.dim;
    const bool mixed = p.precision == PFMG_MIXED;
    const bool jac = p.smoother == PFMG_SMOOTH_JACOBI;
    auto f64 = [&](int n) -> double * {
        char *c = take((size_t)field_stride(n, dim, 8) * 8);
        return c ? (double *)c + field_lead(8) : nullptr;
    };
    auto f32 = [&](int n) -> float * {
        char *c = take((size_t)field_stride(n, dim, 4) * 4);
        return c ? (float *)c + field_lead(4) : nullptr;
    };
    PLevel tmp;
    PLevel &L0 = sv ? sv->L[0] : tmp;
    L0.n = p.n;
    L0.fs = field_stride(p.n, dim, 8);
    L0.mg.clear();
    for (int l = 0, n = p.n;; ++l, n = coarser(n)) {
        MGLevel G;
        G.n = n;
        G.fs64 = field_stride(n, dim, 8);
        G.fs32 = field_stride(n, dim, 4);
        if (l > 0) {
            G.e = {f64(n), G.fs64};
            G.b = {f64(n), G.fs64};
        }
        const bool pingpong = jac || (dim == 3 && n >= 31) || (l == 0 && p.stencil_order == 4);
        if (pingpong) G.t = {f64(n), G.fs64};
        if (mixed) {
            G.e32 = {f32(n), G.fs32};
            G.b32 = {f32(n), G.fs32};
            if (pingpong) G.t32 = {f32(n), G.fs32};
        }
        if (sv) L0.mg.push_back(G);
        if (n <= 2) break;
    }
    double *vb = f64(p.n), *vu = f64(p.n);
    auto *bits = (unsigned long long *)take((size_t)4 * k::RSLOTS * 8);
    int *mask = (int *)take(sizeof(int));
    if (sv) {
        sv->vb = vb;
        sv->vu = vu;
        sv->bits = bits;
        sv->mask = mask;
    }
    return (off + 255) & ~(size_t)255;
}

bool Solver::init_host(std::string &why)
{
    const char *e = getenv("PFMG_NO_XCD_REMAP");
    noremap = (e && atoi(e)) ? 1 : 0;
    e = getenv("PFMG_NO_BOTTOM");
    use_bottom = !(e && atoi(e));
    e = getenv("PFMG_NO_GRAPH");
    graphs = !(e && atoi(e));
    e = getenv("PFMG_FUSED_MIN");
    fused_min_points = e ? atol(e) : 2000000;
    dim = p.dim;
    P = p.n_slices;
    // slice groups of the pipelined iteration: four groups of (nearly)
    // equal size for P >= 8, so that the coarse chain of one group runs
    // under the fine sweeps of the next ones while the fine launches stay
    // large enough to stream well (measured at 127^3 x 16: 4 x 4 slices
    // 1.60 s per block, halving sizes 8,4,2,2 1.66 s, 2 x 8 1.67 s).
    // PFMG_GROUPS: a count of equal groups, or a comma-separated list of
    // group sizes.
    gbound.assign(1, 0);
    // PFMG_FINE_STREAMS=2 alternates the groups' fine sweeps over two
    // streams.  Measured at 127^3 x 16 in four groups it is slower (1.82 s
    // per block against 1.52 s): overlapping fine sweeps delay the first
    // group, and the coarse chain behind it, more than they hide.
    e = getenv("PFMG_FINE_STREAMS");
    fine_streams = e ? std::max(1, atoi(e)) : 1;
    // PFMG_LATE_INTERP=0: each group's interpolation and residual follow
    // its coarse chain on the chain stream (the earlier schedule).
    e = getenv("PFMG_LATE_INTERP");
    late_interp = !(e && atoi(e) == 0);
    // PFMG_ONE_STREAM=1: the pipelined iteration's coarse chain runs on the
    // main stream (for timing kernels without the chain beside them)
    e = getenv("PFMG_ONE_STREAM");
    one_stream = e && atoi(e) != 0;
    // PFMG_FUSED_SDC=0: the separate integral, right-hand-side, F and copy
    // launches of a sweep.
    e = getenv("PFMG_FUSED_SDC");
    fused_sdc = !(e && atoi(e) == 0);
    e = getenv("PFMG_GROUPS");
    if (e && strchr(e, ',')) {
        for (const char *c = e; *c;) {
            const int sz = atoi(c);
            if (sz > 0 && gbound.back() < P) gbound.push_back(std::min(P, gbound.back() + sz));
            c = strchr(c, ',');
            if (!c) break;
            ++c;
        }
        if (gbound.back() < P) gbound.push_back(P);
    } else if (e) {
        const int g = std::max(1, std::min(atoi(e), P));
        for (int q = 1; q <= g; ++q) gbound.push_back((int)((long)P * q / g));
    } else if (P >= 8) {
        for (int q = 1; q <= 4; ++q) gbound.push_back((int)((long)P * q / 4));
    } else {
        gbound.push_back(P);
    }
    if ((int)gbound.size() - 1 > MAXGROUPS) gbound = {0, P};
    groups = (int)gbound.size() - 1;
    nl = levels(p);
    // the pipelined schedule is built for two levels
    if (nl == 3) {
        gbound = {0, P};
        groups = 1;
    }
    for (int lev = 0; lev < nl; ++lev) {
        PLevel &Lv = L[lev];
        const int nn = level_nodes(p, lev);
        if (!family_nodes_ld(p.node_family, nn, Lv.s_ld)) { why = "node construction failed"; return false; }
        for (int q = 0; q < nn; ++q) Lv.s[q] = (double)Lv.s_ld[q];
        if (!collocation_matrices(nn, Lv.s_ld, Lv.Q, Lv.S, Lv.d, p.node_family == PFMG_NODES_UNIFORM ? 1 : 0)) {
            why = "Q construction failed"; return false;
        }
    }
    // (the workspace is carved after this, so node counts come from p)
    for (int l = 0; l + 1 < nl; ++l) {
        for (int mc = 0; mc < level_nodes(p, l + 1); ++mc) {
            cmap[l][mc] = -1;
            for (int mf = 0; mf < level_nodes(p, l); ++mf)
                if (std::fabs((double)(L[l].s_ld[mf] - L[l + 1].s_ld[mc])) < 1e-14) cmap[l][mc] = mf;
            if (cmap[l][mc] < 0) { why = "a level's nodes must be a subset of the finer level's"; return false; }
        }
    }
    return true;
}

hipError_t Solver::upload_constants()
{
    static thread_local double Lt[256];
    for (int lev = 0; lev < nl; ++lev) {
        HC(hipMemcpyAsync(L[lev].dQ, L[lev].Q, sizeof(double) * L[lev].nn * L[lev].nn, hipMemcpyHostToDevice, s));
        HC(hipMemcpyAsync(L[lev].dS, L[lev].S, sizeof(double) * L[lev].nn * L[lev].nn, hipMemcpyHostToDevice, s));
    }
    for (int l = 0; l + 1 < nl; ++l) {
        const int nf = level_nodes(p, l), nc = level_nodes(p, l + 1);
        lagrange_interp(nf, L[l].s_ld, nc, L[l + 1].s_ld, Lt);
        HC(hipMemcpyAsync(dLt[l], Lt, sizeof(double) * nf * nc, hipMemcpyHostToDevice, s));
        // the copy reads the host table when it runs
        HC(hipStreamSynchronize(s));
    }
    return hipStreamSynchronize(s);
}

// ------------------------------------------------------------------ timing
void Timer::start(const char *fam, int n, double bytes_per_point, long points, bool stamped_launch, hipStream_t s)
{
    const int d = depth++;
    if (!on || open >= 0) return;
    if (key != std::string(fam) + "@" + std::to_string(n) || used + 2 > ev.size()) return;
    stamped = stamped_launch;
    added = bytes_per_point * (double)points;
    if (stamped) armed_events = {ev[used], ev[used + 1]};
    else (void)hipEventRecord(ev[used], s);
    bytes += added;
    launches += 1;
    used += 1;
    open = d;
}

void Timer::stop(hipStream_t s)
{
    const int d = --depth;
    if (open != d) return;
    open = -1;
    if (stamped) {
        if (armed_events.start) {              // nothing was launched
            armed_events = {};
            used -= 1;
            launches -= 1;
            bytes -= added;
            return;
        }
    } else {
        (void)hipEventRecord(ev[used], s);
    }
    used += 1;
}

hipError_t Timer::enable(const char *kernel, bool en)
{
    on = en;
    used = 0;
    depth = 0;
    open = -1;
    bytes = 0;
    launches = 0;
    if (!on) return hipSuccess;
    if (!kernel) return hipErrorInvalidValue;
    key = kernel;
    if (ev.empty()) {
        ev.resize(1 << 16);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
    }
    return hipSuccess;
}

hipError_t Timer::read(long long *nl, double *ms, double *nbytes)
{
    double tot = 0;
    for (size_t q = 0; q + 1 < used; q += 2) {
        float e = 0;
        const hipError_t r = hipEventElapsedTime(&e, ev[q], ev[q + 1]);
        if (r != hipSuccess) return r;
        tot += e;
    }
    if (nl) *nl = launches;
    if (ms) *ms = tot;
    if (nbytes) *nbytes = bytes;
    return hipSuccess;
}

void Timer::release()
{
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
}

void Solver::tstart(const char *fam, int n, double bytes_per_point, long points, bool stamped)
{
    timer.start(fam, n, bytes_per_point, points, stamped, s);
}

void Solver::tstop() { timer.stop(s); }

// ------------------------------------------------------------- multigrid
template <typename T>
hipError_t Solver::smooth(int n, int count, const int *m, double alpha, View<T> u, View<T> b, View<T> tmp,
                          int sweeps, bool from_zero)
{
    const Tiling t = tl(n, count, m);
    const double om = p.omega;
    const long pts = interior_points(n, dim) * count;
    const double w = (double)sizeof(T);
    if (sweeps == 0) return from_zero ? k::zero(t, u, s) : hipSuccess;
    // The one-pass sweep marches in z; on small batches (the coarse chain
    // sweeps one slice at a time) its serial steps can cost more than the
    // second pass of the colour-by-colour kernels.  The tuner times both (and
    // the one-pass shapes) on first use; without timing, big batches take
    // the one-pass kernel.
    RbPlan plan;
    if (p.smoother == PFMG_SMOOTH_RBGS && dim == 3 && n >= 31 && n <= 255 && tmp.p) {
        const bool big = (long)count * interior_points(n, dim) >= fused_min_points;
        if (tune) {
            plan = rb_plan<T>(t, alpha, om, b, u, tmp, s, big);
        } else {
            plan.fused = big;
            if (big) plan.shape = k::rbgs_fused_shape(t, sizeof(T));
        }
    }
    if (plan.fused) {
        // whole sweeps in one pass each, ping-pong between u and tmp
        View<T> src = u, dst = tmp;
        for (int q = 0; q < sweeps; ++q) {
            tstart("rbgs", n, 3 * w, pts, true);
            HC(k::rbgs_fused(t, alpha, om, q == 0 && from_zero, b, src, dst, s, &plan.shape));
            tstop();
            std::swap(src, dst);
        }
        if (src.p != u.p) HC(k::copy(t, src, u, s));
        return hipSuccess;
    }
    if (p.smoother == PFMG_SMOOTH_RBGS) {
        for (int q = 0; q < sweeps; ++q) {
            tstart("rbgs", n, 2 * w, pts, true);
            if (q == 0 && from_zero) HC(k::rbgs_zero_red(t, alpha, om, b, u, s));
            else HC(k::rbgs(t, alpha, om, 0, b, u, s));
            tstop();
            tstart("rbgs", n, 2 * w, pts, true);
            HC(k::rbgs(t, alpha, om, 1, b, u, s));
            tstop();
        }
        return hipSuccess;
    }
    View<T> src = u, dst = tmp;
    for (int q = 0; q < sweeps; ++q) {
        tstart("jacobi", n, 3 * w, pts, true);
        if (q == 0 && from_zero) HC(k::jacobi_zero(t, alpha, om, b, dst, s));
        else HC(k::jacobi(t, alpha, om, b, src, dst, s));
        tstop();
        std::swap(src, dst);
    }
    if (src.p != u.p) HC(k::copy(t, src, u, s));
    return hipSuccess;
}

// The fine PFASST level's operator with stencil_order 4: smoothing and the
// residual use L4 on the finest multigrid level, and the correction
// equation below it is the second-order cycle.
hipError_t Solver::vcycle4(int lev, View<double> u, View<double> b, int count, const int *m, double alpha)
{
    if (L[lev].mg.size() < 2) return hipErrorInvalidValue;
    MGLevel &G = L[lev].mg[0];
    MGLevel &C = L[lev].mg[1];
    const Tiling t = tl(G.n, count, m);
    const View<double> gt = scr(G.t), ce = scr(C.e), cb = scr(C.b);
    if (!gt.p || !ce.p || !cb.p) return hipErrorInvalidValue;
    HC(smooth4(t, alpha, u, b, gt, p.nu_pre));
    HC(k::resid4(t, alpha, b, u, gt, s));
    HC(k::restrict_fw(t, gt, cb, s));
    HC(vcycle64(lev, 1, ce, cb, count, m, alpha));
    HC(k::prolong_add(t, ce, u, s));
    return smooth4(t, alpha, u, b, gt, p.nu_post);
}

// Sweeps of weighted Jacobi (every point, then copied back) or red-black
// JOR (red from u into tmp, black from tmp back into u).
hipError_t Solver::smooth4(const Tiling &t, double alpha, View<double> u, View<double> b, View<double> tmp, int sweeps)
{
    for (int q = 0; q < sweeps; ++q) {
        if (p.smoother == PFMG_SMOOTH_RBGS) {
            HC(k::smooth4(t, alpha, p.omega, 0, b, u, tmp, s));
            HC(k::smooth4(t, alpha, p.omega, 1, b, tmp, u, s));
        } else {
            HC(k::smooth4(t, alpha, p.omega, -1, b, u, tmp, s));
            HC(k::copy(t, tmp, u, s));
        }
    }
    return hipSuccess;
}

hipError_t Solver::resid_norm_lev(int lev, const Tiling &t, double alpha, View<double> b, View<double> u,
                                  unsigned long long *out)
{
    if (lev == 0 && p.stencil_order == 4) {
        const View<double> r = scr(L[0].mg[0].t);
        if (!r.p) return hipErrorInvalidValue;
        HC(k::resid4(t, alpha, b, u, r, s));
        return k::norm_inf(t, r, out, s);
    }
    return k::resid_norm(t, alpha, b, u, out, s);
}

hipError_t Solver::apply_F(int lev, const Tiling &t, View<double> u, View<double> F)
{
    if (lev == 0 && p.stencil_order == 4) return k::apply_L4(t, p.nu, u, F, s);
    return k::apply_L(t, p.nu, u, F, s);
}

hipError_t Solver::vcycle64(int lev, int l, View<double> u, View<double> b, int count, const int *m, double alpha)
{
    if (lev == 0 && l == 0 && p.stencil_order == 4) return vcycle4(lev, u, b, count, m, alpha);
    MGLevel &G = L[lev].mg[l];
    const Tiling t = tl(G.n, count, m);
    if (use_bottom && k::vcycle_bottom_lds(G.n, dim, p.smoother, sizeof(double)) <= k::bottom_lds_max())
        return k::vcycle_bottom(t, alpha, p.smoother, p.omega, p.nu_pre, p.nu_post, l > 0, b, u, s);
    if (G.n <= 2) return k::coarsest(t, alpha, b, u, s);
    const View<double> gt = scr(G.t);
    HC(smooth<double>(G.n, count, m, alpha, u, b, gt, p.nu_pre, l > 0));
    MGLevel &C = L[lev].mg[l + 1];
    const View<double> ce = scr(C.e), cb = scr(C.b);
    const long pts = interior_points(G.n, dim) * count;
    tstart("resid_restrict", G.n, 16 + 8.0 / (dim == 3 ? 8 : 2), pts);
    HC(k::resid_restrict(t, alpha, b, u, cb, s));
    tstop();
    HC(vcycle64(lev, l + 1, ce, cb, count, m, alpha));
    tstart("prolong", G.n, 16 + 8.0 / (dim == 3 ? 8 : 2), pts);
    HC(k::prolong_add(t, ce, u, s));
    tstop();
    return smooth<double>(G.n, count, m, alpha, u, b, gt, p.nu_post, false);
}

hipError_t Solver::vcycle32(int lev, int l, View<float> u, View<float> b, int count, const int *m, double alpha)
{
    MGLevel &G = L[lev].mg[l];
    const Tiling t = tl(G.n, count, m);
    if (use_bottom && k::vcycle_bottom_lds(G.n, dim, p.smoother, sizeof(float)) <= k::bottom_lds_max())
        return k::vcycle_bottom(t, alpha, p.smoother, p.omega, p.nu_pre, p.nu_post, true, b, u, s);
    if (G.n <= 2) return k::coarsest(t, alpha, b, u, s);
    const View<float> gt = scr(G.t32);
    HC(smooth<float>(G.n, count, m, alpha, u, b, gt, p.nu_pre, true));
    MGLevel &C = L[lev].mg[l + 1];
    const View<float> ce = scr(C.e32), cb = scr(C.b32);
    HC(k::resid_restrict(t, alpha, b, u, cb, s));
    HC(vcycle32(lev, l + 1, ce, cb, count, m, alpha));
    HC(k::prolong_add(t, ce, u, s));
    return smooth<float>(G.n, count, m, alpha, u, b, gt, p.nu_post, false);
}

// One V-cycle, or one refinement step of the mixed form: FP64 residual
// rounded to FP32, FP32 V-cycle from a zero correction, FP64 update.
hipError_t Solver::cycle_step(int lev, View<double> u, View<double> b, int count, const int *m, double alpha)
{
    if (p.precision != PFMG_MIXED) return vcycle64(lev, 0, u, b, count, m, alpha);
    MGLevel &G = L[lev].mg[0];
    const Tiling t = tl(G.n, count, m);
    const View<float> ge = scr(G.e32), gb = scr(G.b32);
    HC(k::resid_round(t, alpha, b, u, gb, s));
    HC(vcycle32(lev, 0, ge, gb, count, m, alpha));
    return k::add_f32(t, ge, u, s);
}

hipError_t Solver::solve(int lev, View<double> u, View<double> b, int count, double alpha, int cycles,
                         double *relres_host)
{
    const int n = L[lev].n;
    last_solve_status = 0;
    if (cycles > 0) {
        for (int c = 0; c < cycles; ++c) {
            // "vcycle@n" brackets whole cycles; its byte counter holds DOF x cycles
            tstart("vcycle", n, 1.0, interior_points(n, dim) * count);
            HC(cycle_step(lev, u, b, count, nullptr, alpha));
            tstop();
        }
        vcount[lev] += (long long)cycles * count;
        if (relres_host) {
            HC(k::fill_u64(bits, 0, 2 * count, s));
            HC(k::norm_inf(tl(n, count), b, bits, s));
            HC(resid_norm_lev(lev, tl(n, count), alpha, b, u, bits + count));
            HC(hipMemcpyAsync(hbits, bits, sizeof(unsigned long long) * 2 * count, hipMemcpyDeviceToHost, s));
            HC(hipStreamSynchronize(s));
            for (int q = 0; q < count; ++q) {
                const double nb = bits_to_double(hbits[q]), r = bits_to_double(hbits[count + q]);
                relres_host[q] = nb > 0 ? r / nb : r;
            }
        }
        return hipSuccess;
    }
    // Full solve, per field: repeat while |r| > tol |b| and each cycle cuts
    // the residual below stall * the previous one, at most mg_max_cycles.
    HC(k::fill_u64(bits, 0, 2 * count, s));
    HC(k::norm_inf(tl(n, count), b, bits, s));
    HC(resid_norm_lev(lev, tl(n, count), alpha, b, u, bits + count));
    HC(hipMemcpyAsync(hbits, bits, sizeof(unsigned long long) * 2 * count, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    std::vector<double> nb(count), rold(count);
    for (int q = 0; q < count; ++q) {
        nb[q] = bits_to_double(hbits[q]);
        rold[q] = bits_to_double(hbits[count + q]);
        if (!std::isfinite(nb[q]) || !std::isfinite(rold[q])) { last_solve_status = PFMG_ERR_NAN; return hipSuccess; }
    }
    // fine-level node solves: record the training pair, try the learned guess
    const bool rec = lev == 0 && rec_pairs && rec_count + count <= rec_cap && dim == 3 && p.stencil_order == 2;
    const bool learned = lev == 0 && unet && p.guess == PFMG_GUESS_LEARNED;
    if (rec || learned) HC(learned_guess(u, b, count, alpha, nb, rold, rec));
    int active = 0;
    for (int q = 0; q < count; ++q) {
        hmask[q] = rold[q] > p.mg_tol * nb[q];
        active += hmask[q];
    }
    int c = 0;
    bool stalled_any = false;
    while (c < p.mg_max_cycles && active > 0) {
        HC(hipMemcpyAsync(mask, hmask, sizeof(int) * count, hipMemcpyHostToDevice, s));
        tstart("vcycle", n, 1.0, interior_points(n, dim) * active);
        HC(cycle_step(lev, u, b, count, mask, alpha));
        tstop();
        ++c;
        vcount[lev] += active;
        HC(k::fill_u64(bits + count, 0, count, s));
        HC(resid_norm_lev(lev, tl(n, count, mask), alpha, b, u, bits + count));
        HC(hipMemcpyAsync(hbits + count, bits + count, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        active = 0;
        for (int q = 0; q < count; ++q) {
            if (!hmask[q]) continue;
            const double rn = bits_to_double(hbits[count + q]);
            if (!std::isfinite(rn)) { last_solve_status = PFMG_ERR_NAN; return hipSuccess; }
            const bool stalled = !(rn < p.mg_stall * rold[q]);
            rold[q] = rn;
            if (rn <= p.mg_tol * nb[q]) hmask[q] = 0;
            else if (stalled) { hmask[q] = 0; stalled_any = true; }
            active += hmask[q];
        }
    }
    if (relres_host)
        for (int q = 0; q < count; ++q) relres_host[q] = nb[q] > 0 ? rold[q] / nb[q] : rold[q];
    if (rec) {
        HC(nn::record_target(tl(n, count), u, nnsc, rec_scratch, rec_pairs, rec_count, s));
        rec_count += count;
    }
    if (stalled_any) last_solve_status = PFMG_STALLED;
    else if (active > 0) last_solve_status = PFMG_NOT_CONVERGED;
    return hipSuccess;
}

// Before the V-cycles of a full fine-level node solve: scale factors
// sr = |b - H u|_inf, su = |u|_inf per field; record the pair's inputs; and
// with an attached network, its guess g = u + sr y replaces u in every field
// where |b - H g|_inf < |b - H u|_inf (the FP64 residual judges).  rold is
// updated for the fields that take the guess.
hipError_t Solver::learned_guess(View<double> u, View<double> b, int count, double alpha,
                                 const std::vector<double> &nb, std::vector<double> &rold, bool rec)
{
    const int n = L[0].n;
    const Tiling t = tl(n, count);
    HC(k::fill_u64(bits + 2 * count, 0, count, s));
    HC(k::norm_inf(t, u, bits + 2 * count, s));
    HC(hipMemcpyAsync(hbits + 2 * count, bits + 2 * count, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    for (int q = 0; q < count; ++q) {
        const double su = bits_to_double(hbits[2 * count + q]);
        hnnsc[q] = rold[q] > 0 ? rold[q] : 1.0;
        hnnsc[count + q] = su > 0 ? su : 1.0;
    }
    HC(hipMemcpyAsync(nnsc, hnnsc, sizeof(double) * 2 * count, hipMemcpyHostToDevice, s));
    if (rec) HC(nn::record_inputs(t, alpha, b, u, nnsc, nnsc + count, rec_pairs, rec_ah2, rec_count, rec_scratch, s));
    if (!(unet && p.guess == PFMG_GUESS_LEARNED)) return hipSuccess;
    // offer the guess only to fields whose plain guess is still far off
    std::vector<char> offer(count);
    int offered = 0;
    for (int q = 0; q < count; ++q) {
        offer[q] = rold[q] > p.guess_min_relres * nb[q];
        offered += offer[q];
    }
    if (offered == 0) return hipSuccess;
    View<double> g = L[0].mg[0].t;
    hipStream_t ns = unet->s;
    unet->s = s;
    hipError_t e = nn::make_input(t, alpha, b, u, nnsc, nnsc + count, unet->x0, s);
    if (e == hipSuccess) e = unet->forward(count);
    unet->s = ns;
    HC(e);
    HC(nn::apply_guess(t, u, unet->y, nnsc, g, s));
    HC(k::fill_u64(bits + count, 0, count, s));
    HC(k::resid_norm(t, alpha, b, g, bits + count, s));
    HC(hipMemcpyAsync(hbits + count, bits + count, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    int taken = 0;
    for (int q = 0; q < count; ++q) {
        const double rg = bits_to_double(hbits[count + q]);
        hmask[q] = offer[q] && std::isfinite(rg) && rg < rold[q];
        if (hmask[q]) rold[q] = rg;
        taken += hmask[q];
    }
    guess_tried += offered;
    guess_taken += taken;
    if (taken == 0) return hipSuccess;
    HC(hipMemcpyAsync(mask, hmask, sizeof(int) * count, hipMemcpyHostToDevice, s));
    return k::copy(tl(n, count, mask), g, u, s);
}

// ------------------------------------------------------------------- SDC
hipError_t Solver::sweep(int lev, int p0, int p1, const double *u0src, const double *f0src, long src_stride)
{
    PLevel &Lv = L[lev];
    const int count = p1 - p0;
    if (count <= 0) return hipSuccess;
    const int nn = Lv.nn;
    const long fs = Lv.fs, sst = (long)nn * fs, ist = (long)(nn - 1) * fs;
    const Tiling t = tl(Lv.n, count);
    const long pts = interior_points(Lv.n, dim) * count;
    View<double> Bv{Lv.B + (long)p0 * fs, fs};
    // views of the right-hand side of node m+1: U[m], F[m+1], I[m], tau
    View<double> Um, Fm1, Im, t1, t0;
    auto rhs_views = [&](int m) {
        Um = {Lv.slot(Lv.U, p0, m), sst};
        Fm1 = {Lv.slot(Lv.F, p0, m + 1), sst};
        Im = {Lv.I + (long)p0 * ist + (long)m * fs, ist};
        t1 = t0 = View<double>{nullptr, 0};
        if (lev >= 1) {
            t1 = {Lv.slot(Lv.Tau, p0, m + 1), sst};
            t0 = {Lv.slot(Lv.Tau, p0, m), sst};
        }
    };
    // A new node 0 taken from a source gets F = nu L_h of its value when
    // the source's F came from a solve (f_solve); sources are coarse nodes.
    const bool eval0 = u0src && p.f_solve;
    if (eval0 && lev == 0) return hipErrorInvalidValue;
    if (fused_sdc) {
        // node 0 from the source, the integrals and the first right-hand side
        const View<double> us{const_cast<double *>(u0src), src_stride};
        const View<double> fsrc{const_cast<double *>(f0src), src_stride};
        tstart("sdc_start", Lv.n, 8.0 * (2 * nn - 1) + 16 + (lev >= 1 ? 16 : 0) + (u0src ? 16 : 0), pts);
        HC(k::sdc_start(t, nn, p.dt, Lv.dS, p.dt * Lv.d[1], View<double>{Lv.slot(Lv.U, p0, 0), sst},
                        View<double>{Lv.slot(Lv.F, p0, 0), sst}, us, fsrc, View<double>{Lv.I + (long)p0 * ist, ist},
                        lev >= 1 ? View<double>{Lv.slot(Lv.Tau, p0, 0), sst} : View<double>{nullptr, 0}, Bv, s,
                        eval0 ? p.nu : 0.0));
        tstop();
    } else {
        if (u0src) {
            HC(k::copy(t, View<double>{const_cast<double *>(u0src), src_stride},
                       View<double>{Lv.slot(Lv.U, p0, 0), sst}, s));
            if (eval0)
                HC(apply_F(lev, t, View<double>{Lv.slot(Lv.U, p0, 0), sst}, View<double>{Lv.slot(Lv.F, p0, 0), sst}));
            else
                HC(k::copy(t, View<double>{const_cast<double *>(f0src), src_stride},
                           View<double>{Lv.slot(Lv.F, p0, 0), sst}, s));
        }
        tstart("sdc_integrals", Lv.n, 8.0 * (2 * nn - 1), pts);
        HC(k::sdc_integrals(t, nn, p.dt, Lv.dS, View<double>{Lv.slot(Lv.F, p0, 0), sst},
                            View<double>{Lv.I + (long)p0 * ist, ist}, s));
        tstop();
        rhs_views(0);
        tstart("sdc_rhs", Lv.n, lev >= 1 ? 48 : 32, pts);
        HC(k::sdc_rhs(t, p.dt * Lv.d[1], Um, Fm1, Im, t1, t0, Bv, s));
        tstop();
    }
    const bool fuse_rhs = fused_sdc && k::apply_L_rhs_ok(t) && !(lev == 0 && p.stencil_order == 4);
    for (int m = 0; m + 1 < nn; ++m) {
        // Bv holds the right-hand side of node m+1
        const double delta = p.dt * Lv.d[m + 1];
        View<double> Uv{Lv.slot(Lv.U, p0, m + 1), sst}, Fv{Lv.slot(Lv.F, p0, m + 1), sst};
        HC(solve(lev, Uv, Bv, count, p.nu * delta, p.vcycles_per_solve, nullptr));
        if (last_solve_status == PFMG_ERR_NAN) return hipSuccess;
        const bool more = m + 2 < nn;
        if (more) rhs_views(m + 1);
        if (p.f_solve) {
            // F from the solve, then the next right-hand side (Um is node m+1)
            tstart("solve_F", Lv.n, more ? (lev >= 1 ? 72 : 56) : 24, pts);
            HC(k::solve_F_rhs(t, delta, Uv, Bv, Fv, more ? p.dt * Lv.d[m + 2] : 0.0,
                              more ? Fm1 : View<double>{nullptr, 0}, more ? Im : View<double>{nullptr, 0},
                              more ? t1 : View<double>{nullptr, 0}, more ? t0 : View<double>{nullptr, 0}, s));
            tstop();
            continue;
        }
        if (more && fuse_rhs) {
            // F of node m+1 and the right-hand side of node m+2, which reads
            // the old F of node m+2, not the new F of node m+1
            tstart("apply_L", Lv.n, 16, pts);
            HC(k::apply_L_rhs(t, p.nu, Uv, Fv, p.dt * Lv.d[m + 2], Fm1, Im, t1, t0, Bv, s));
            tstop();
            continue;
        }
        tstart("apply_L", Lv.n, 16, pts);
        HC(apply_F(lev, t, Uv, Fv));
        tstop();
        if (more) {
            tstart("sdc_rhs", Lv.n, lev >= 1 ? 48 : 32, pts);
            HC(k::sdc_rhs(t, p.dt * Lv.d[m + 2], Um, Fm1, Im, t1, t0, Bv, s));
            tstop();
        }
    }
    return hipSuccess;
}

// Level l to l+1; below the middle level the finer level's own FAS term
// joins the restricted integrals (tau_c = R(dt Q_f F_f + tau_f) - dt Q_c F_c).
hipError_t Solver::fas_restrict(int p0, int p1, int l)
{
    PLevel &Fn = L[l], &Cs = L[l + 1];
    const int count = p1 - p0;
    const long fst = (long)Fn.nn * Fn.fs, cst = (long)Cs.nn * Cs.fs;
    HC(k::fas_inject(tl(Cs.n, count), Fn.nn, Cs.nn, cmap[l], p.dt, Fn.dQ,
                     View<double>{Fn.slot(Fn.U, p0, 0), fst}, View<double>{Fn.slot(Fn.F, p0, 0), fst},
                     View<double>{Cs.slot(Cs.U, p0, 0), cst}, View<double>{Cs.slot(Cs.Uold, p0, 0), cst},
                     View<double>{Cs.slot(Cs.Tau, p0, 0), cst}, s,
                     l > 0 ? View<double>{Fn.slot(Fn.Tau, p0, 0), fst} : View<double>{nullptr, 0}));
    HC(k::apply_L(tl(Cs.n, count * Cs.nn), p.nu, View<double>{Cs.slot(Cs.U, p0, 0), Cs.fs},
                  View<double>{Cs.slot(Cs.F, p0, 0), Cs.fs}, s));
    if (Cs.Fold)
        HC(k::copy(tl(Cs.n, count * Cs.nn), View<double>{Cs.slot(Cs.F, p0, 0), Cs.fs},
                   View<double>{Cs.slot(Cs.Fold, p0, 0), Cs.fs}, s));
    return k::fas_tau(tl(Cs.n, count), Cs.nn, p.dt, Cs.dQ, View<double>{Cs.slot(Cs.F, p0, 0), cst},
                      View<double>{Cs.slot(Cs.Tau, p0, 0), cst}, s);
}

hipError_t Solver::interpolate(int p0, int p1, int l)
{
    PLevel &Fn = L[l], &Cs = L[l + 1];
    const double *dLt = this->dLt[l];
    const int count = p1 - p0;
    const long cst = (long)Cs.nn * Cs.fs, dst = (long)Fn.nn * Cs.fs;
    double *dc = Cs.DC + (long)p0 * dst;
    HC(k::interp_coarse(tl(Cs.n, count), Fn.nn, Cs.nn, dLt, View<double>{Cs.slot(Cs.U, p0, 0), cst},
                        View<double>{Cs.slot(Cs.Uold, p0, 0), cst}, View<double>{dc, dst}, s));
    const long pts = interior_points(Fn.n, dim) * count * Fn.nn;
    if (p.f_interp && p.interp_order == 4) {
        // the coarse F change beside U's, and both cubic interpolations in
        // one launch (shared indices and weights)
        double *dcf = Cs.DCF + (long)p0 * dst;
        HC(k::interp_coarse(tl(Cs.n, count), Fn.nn, Cs.nn, dLt, View<double>{Cs.slot(Cs.F, p0, 0), cst},
                            View<double>{Cs.slot(Cs.Fold, p0, 0), cst}, View<double>{dcf, dst}, s));
        tstart("prolong", Fn.n, 32 + 16.0 / (dim == 3 ? 8 : 2), pts);
        HC(k::prolong4_add2(tl(Fn.n, count * Fn.nn), View<double>{dc, Cs.fs}, View<double>{Fn.slot(Fn.U, p0, 0), Fn.fs},
                            View<double>{dcf, Cs.fs}, View<double>{Fn.slot(Fn.F, p0, 0), Fn.fs}, s));
        tstop();
        return hipSuccess;
    }
    tstart("prolong", Fn.n, 16 + 8.0 / (dim == 3 ? 8 : 2), pts);
    if (p.interp_order == 4)
        HC(k::prolong4_add(tl(Fn.n, count * Fn.nn), View<double>{dc, Cs.fs}, View<double>{Fn.slot(Fn.U, p0, 0), Fn.fs}, s));
    else
        HC(k::prolong_add(tl(Fn.n, count * Fn.nn), View<double>{dc, Cs.fs}, View<double>{Fn.slot(Fn.U, p0, 0), Fn.fs}, s));
    tstop();
    if (p.f_interp) {
        // the coarse F change, interpolated in time and space like U's
        HC(k::interp_coarse(tl(Cs.n, count), Fn.nn, Cs.nn, dLt, View<double>{Cs.slot(Cs.F, p0, 0), cst},
                            View<double>{Cs.slot(Cs.Fold, p0, 0), cst}, View<double>{dc, dst}, s));
        tstart("prolong", Fn.n, 16 + 8.0 / (dim == 3 ? 8 : 2), pts);
        if (p.interp_order == 4)
            HC(k::prolong4_add(tl(Fn.n, count * Fn.nn), View<double>{dc, Cs.fs}, View<double>{Fn.slot(Fn.F, p0, 0), Fn.fs}, s));
        else
            HC(k::prolong_add(tl(Fn.n, count * Fn.nn), View<double>{dc, Cs.fs}, View<double>{Fn.slot(Fn.F, p0, 0), Fn.fs}, s));
        tstop();
        return hipSuccess;
    }
    tstart("apply_L", Fn.n, 16, pts);
    HC(apply_F(l, tl(Fn.n, count * Fn.nn), View<double>{Fn.slot(Fn.U, p0, 0), Fn.fs},
               View<double>{Fn.slot(Fn.F, p0, 0), Fn.fs}));
    tstop();
    return hipSuccess;
}

hipError_t Solver::spread(const double *u0_dev)
{
    PLevel &Fn = L[0];
    HC(k::unpack(tl(Fn.n, 1), u0_dev, View<double>{ublock, 0}, s));
    if (use_graph() && warm_start) {
        if (!g_start) HC(capture([this] { return spread_body(); }, &g_start, vc_start));
        for (int l = 0; l < 3; ++l) vcount[l] += vc_start[l];
        return hipGraphLaunch(g_start, s);
    }
    // the first block start runs eagerly: launch shapes are tuned outside
    // capture, and the captured graph replays the tuned launches
    warm_start = true;
    return spread_body();
}

// Everything of a block start after u_block is in place: spread to all nodes
// and slices, F, the injected coarse initial value and the predictor.
hipError_t Solver::spread_body()
{
    PLevel &Fn = L[0];
    HC(k::copy(tl(Fn.n, P * Fn.nn), View<double>{ublock, 0}, View<double>{Fn.U, Fn.fs}, s));
    HC(apply_F(0, tl(Fn.n, P * Fn.nn), View<double>{ublock, 0}, View<double>{Fn.F, Fn.fs}));
    if (nl == 2) HC(k::inject(tl(L[1].n, 1), View<double>{ublock, 0}, View<double>{ublock_c, 0}, s));
    if (nl == 3) {
        HC(k::inject(tl(L[1].n, 1), View<double>{ublock, 0}, View<double>{ublock_m, 0}, s));
        HC(k::inject(tl(L[2].n, 1), View<double>{ublock_m, 0}, View<double>{ublock_c, 0}, s));
    }
    if (nl > 1)
        HC(k::apply_L(tl(L[nl - 1].n, 1), p.nu, View<double>{ublock_c, 0}, View<double>{fublock_c, 0}, s));
    HC(predictor());
    return snapshot_ends(0, P);
}

// AFTER_SWEEP: keep the fine end values of slices p0 .. p1-1 as the values
// they send at the next iteration.
hipError_t Solver::snapshot_ends(int p0, int p1)
{
    if (!esnap || p1 <= p0) return hipSuccess;
    PLevel &Fn = L[0];
    return k::copy(tl(Fn.n, p1 - p0), View<double>{Fn.slot(Fn.U, p0, Fn.nn - 1), (long)Fn.nn * Fn.fs},
                   View<double>{esnap + (long)p0 * Fn.fs, Fn.fs}, s);
}

// Predictor (Sec. 2.4): round j sweeps every slice p >= j on the coarse
// level; for j >= 1 those slices first take slice p-1's end value of round
// j-1 (all copies precede the round's sweeps, so no snapshot is needed).
hipError_t Solver::predictor()
{
    if (nl < 2) return hipSuccess;
    const int Lc = nl - 1;
    PLevel &Cs = L[Lc];
    const int Mc = Cs.nn - 1;
    const long cst = (long)Cs.nn * Cs.fs;
    for (int l = 0; l < Lc; ++l) HC(fas_restrict(0, P, l));
    for (int j = 0; j < P; ++j) {
        // round j >= 1: slices j .. P-1 first take node 0 from the previous
        // slice's last node (in the sweep's first kernel)
        if (j >= 1) HC(sweep(Lc, j, P, Cs.slot(Cs.U, j - 1, Mc), Cs.slot(Cs.F, j - 1, Mc), cst));
        else HC(sweep(Lc, j, P));
        if (last_solve_status == PFMG_ERR_NAN) return hipSuccess;
    }
    // straight up, without middle-level sweeps
    for (int l = Lc - 1; l >= 0; --l) HC(interpolate(0, P, l));
    return hipSuccess;
}

// Per-slice maxima land in RSLOTS partial slots per slice (spreading the
// atomics); the host takes the maximum over the slots.
hipError_t Solver::residual_enqueue()
{
    HC(k::fill_u64(bits, 0, 2 * P * k::RSLOTS, s));
    return residual_slices(0, P);
}

// Residual partials of slices p0 .. p1-1 (bits cleared beforehand); slice
// p0 > 0 takes its initial value from slice p0-1's last node.
hipError_t Solver::residual_slices(int p0, int p1)
{
    PLevel &Fn = L[0];
    const long fst = (long)Fn.nn * Fn.fs;
    const int count = p1 - p0;
    double *Fr = Fn.F;
    if (Fn.Ft) {
        // the stored F is not F(U) mid-iteration: evaluate F(U) for eq. resid
        tstart("apply_L", Fn.n, 16, interior_points(Fn.n, dim) * count * Fn.nn);
        HC(apply_F(0, tl(Fn.n, count * Fn.nn), View<double>{Fn.U + (long)p0 * fst, Fn.fs},
                   View<double>{Fn.Ft + (long)p0 * fst, Fn.fs}));
        tstop();
        Fr = Fn.Ft;
    }
    tstart("colloc_resid", Fn.n, 8.0 * (2 * Fn.nn + 1), interior_points(Fn.n, dim) * count);
    HC(k::colloc_resid(tl(Fn.n, count), Fn.nn, P, p.dt, Fn.dQ, View<double>{Fn.U + (long)p0 * fst, fst},
                       View<double>{Fr + (long)p0 * fst, fst}, View<double>{ublock, 0},
                       bits + (long)p0 * k::RSLOTS, bits + (long)(P + p0) * k::RSLOTS, s, p0));
    tstop();
    return hipSuccess;
}

hipError_t Solver::residual_read(double *per_slice, double *block)
{
    const int ns = 2 * P * k::RSLOTS;
    HC(hipMemcpyAsync(hbits, bits, sizeof(unsigned long long) * ns, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    double blk = 0;
    bool bad = false;
    for (int q = 0; q < P; ++q) {
        unsigned long long rb = 0, ub = 0;
        for (int w = 0; w < k::RSLOTS; ++w) {
            rb = std::max(rb, hbits[(long)q * k::RSLOTS + w]);
            ub = std::max(ub, hbits[(long)(P + q) * k::RSLOTS + w]);
        }
        const double r = bits_to_double(rb), u0 = bits_to_double(ub);
        const double v = p.residual_abs || !(u0 > 0) ? r : r / u0;
        if (!std::isfinite(v)) bad = true;
        if (per_slice) per_slice[q] = v;
        if (v > blk || v != v) blk = v;
    }
    if (block) *block = blk;
    last_solve_status = bad ? PFMG_ERR_NAN : 0;
    return hipSuccess;
}

hipError_t Solver::residual(double *per_slice, double *block)
{
    HC(residual_enqueue());
    return residual_read(per_slice, block);
}

hipError_t Solver::iterate_body()
{
    PLevel &Fn = L[0];
    const int M = Fn.nn - 1;
    const long fst = (long)Fn.nn * Fn.fs;
    // new fine initial values from the previous iteration's end values, all
    // slices at once, before any sweep changes them
    if (P > 1) {
        // the sent values: the end values now, or those kept after the last
        // fine sweeps (AFTER_SWEEP)
        const View<double> sent = esnap ? View<double>{esnap, Fn.fs} : View<double>{Fn.slot(Fn.U, 0, M), fst};
        HC(k::copy(tl(Fn.n, P - 1), sent, View<double>{Fn.slot(Fn.U, 1, 0), fst}, s));
        // F of the new node 0: the sent F is F(U) unless it came from a
        // solve or an interpolation, or was kept before the correction
        if (p.f_solve || p.f_interp || esnap)
            HC(apply_F(0, tl(Fn.n, P - 1), View<double>{Fn.slot(Fn.U, 1, 0), fst}, View<double>{Fn.slot(Fn.F, 1, 0), fst}));
        else
            HC(k::copy(tl(Fn.n, P - 1), View<double>{Fn.slot(Fn.F, 0, M), fst}, View<double>{Fn.slot(Fn.F, 1, 0), fst}, s));
    }
    if (nl == 2 && groups > 1 && p.vcycles_per_solve > 0) return iterate_pipelined();
    HC(sweep(0, 0, P));
    if (last_solve_status == PFMG_ERR_NAN) return hipSuccess;
    HC(snapshot_ends(0, P));
    if (nl > 1) {
        const int Lc = nl - 1;
        for (int l = 0; l < Lc; ++l) {
            HC(fas_restrict(0, P, l));
            // a middle level sweeps on the way down
            if (l + 1 < Lc) {
                HC(sweep(l + 1, 0, P));
                if (last_solve_status == PFMG_ERR_NAN) return hipSuccess;
            }
        }
        for (int q = 0; q < P; ++q) {
            HC(chain_step(q));
            if (last_solve_status == PFMG_ERR_NAN) return hipSuccess;
        }
        for (int l = Lc - 1; l >= 0; --l) {
            HC(interpolate(0, P, l));
            // and on the way up
            if (l > 0) {
                HC(sweep(l, 0, P));
                if (last_solve_status == PFMG_ERR_NAN) return hipSuccess;
            }
        }
    }
    return residual_enqueue();
}

// Coarse sweep of slice q with its new initial value: the block's injected
// initial value for q = 0, else slice q-1's end value of this iteration.
hipError_t Solver::chain_step(int q)
{
    const int Lc = nl - 1;
    PLevel &Cs = L[Lc];
    const int Mc = Cs.nn - 1;
    const double *us = q == 0 ? ublock_c : Cs.slot(Cs.U, q - 1, Mc);
    const double *fsrc = q == 0 ? fublock_c : Cs.slot(Cs.F, q - 1, Mc);
    return sweep(Lc, q, q + 1, us, fsrc, 0);
}

// The same iteration with the slices in groups: the fine sweep and FAS
// restriction of group g run on the main stream while the coarse chain of
// the earlier groups runs on a second stream (chain step q needs only slice
// q's restriction and slice q-1's coarse end value, and interpolation of a
// group only its own coarse sweeps).  Every slice sees the same operations
// in the same order as in the sequential schedule.  Fixed V-cycle counts
// only (full solves read norms back on the host).
hipError_t Solver::iterate_pipelined()
{
    if (!s2) HC(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    for (int g = 0; g <= groups; ++g)
        if (!ev[g]) HC(hipEventCreateWithFlags(&ev[g], hipEventDisableTiming));
    const int G = groups;
    // one_stream: the chain goes to the main stream behind the fine sweeps
    // (the same launches in the same per-slice order, without overlap)
    hipStream_t const s2 = one_stream ? s : this->s2;
    auto first = [&](int g) { return gbound[g]; };
    // The fine sweeps of the groups touch disjoint slices and, with the
    // multigrid scratch offset to their first slice, disjoint scratch, so
    // they may alternate over two streams (fine_streams = 2).
    hipStream_t main = s;
    HC(k::fill_u64(bits, 0, 2 * P * k::RSLOTS, main));   // residual partials, filled per group below
    const int nfs = fine_streams > 1 && G > 1 ? 2 : 1;
    if (nfs > 1) {
        if (!s3) HC(hipStreamCreateWithFlags(&s3, hipStreamNonBlocking));
        if (!ev_fork) HC(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        HC(hipEventRecord(ev_fork, main));
        HC(hipStreamWaitEvent(s3, ev_fork, 0));
    }
    for (int g = 0; g < G; ++g) {
        s = (nfs > 1 && (g & 1)) ? s3 : main;
        mg_off = first(g);
        hipError_t e = sweep(0, first(g), first(g + 1));
        if (e == hipSuccess) e = snapshot_ends(first(g), first(g + 1));
        if (e == hipSuccess) e = fas_restrict(first(g), first(g + 1));
        if (e == hipSuccess) e = hipEventRecord(ev[g], s);
        s = main;
        mg_off = 0;
        HC(e);
    }
    s = s2;
    hipError_t e = hipSuccess;
    if (!late_interp) {
        // each group's collocation residual follows its interpolation (its
        // first slice reads the previous group's end value, interpolated
        // before), so only the last group's is left after the fine sweeps
        for (int g = 0; g < G && e == hipSuccess; ++g) {
            e = hipStreamWaitEvent(s2, ev[g], 0);
            for (int q = first(g); q < first(g + 1) && e == hipSuccess; ++q) e = chain_step(q);
            if (e == hipSuccess) e = interpolate(first(g), first(g + 1));
            if (e == hipSuccess) e = residual_slices(first(g), first(g + 1));
        }
        if (e == hipSuccess) e = hipEventRecord(ev[G], s2);
        s = main;
        HC(e);
        return hipStreamWaitEvent(s, ev[G], 0);
    }
    // Interpolation and residual stream through HBM and would slow the fine
    // sweeps they overlap by about their own duration; the coarse chain is
    // latency-bound and leaves HBM mostly idle.  So the chain stream runs
    // the chain alone, and the main stream, once its last fine sweep is
    // done, interpolates groups 0 .. G-2 (one launch each) while the last
    // group's chain runs, then the last group.
    for (int i = 0; i < 2; ++i)
        if (!evc[i]) HC(hipEventCreateWithFlags(&evc[i], hipEventDisableTiming));
    for (int g = 0; g < G && e == hipSuccess; ++g) {
        e = hipStreamWaitEvent(s2, ev[g], 0);
        for (int q = first(g); q < first(g + 1) && e == hipSuccess; ++q) e = chain_step(q);
        if (e == hipSuccess && g >= G - 2) e = hipEventRecord(evc[g - (G - 2)], s2);
    }
    s = main;
    HC(e);
    // the residual of a group's first slice reads the previous group's end
    // value: interpolation of groups 0 .. G-2 comes before the last residual
    HC(hipStreamWaitEvent(main, evc[0], 0));
    HC(interpolate(0, first(G - 1)));
    HC(residual_slices(0, first(G - 1)));
    HC(hipStreamWaitEvent(main, evc[1], 0));
    HC(interpolate(first(G - 1), P));
    return residual_slices(first(G - 1), P);
}

hipError_t Solver::iterate(double *block)
{
    if (use_graph() && warm_iter) {
        if (!g_iter) HC(capture([this] { return iterate_body(); }, &g_iter, vc_iter));
        for (int l = 0; l < 3; ++l) vcount[l] += vc_iter[l];
        HC(hipGraphLaunch(g_iter, s));
    } else {
        warm_iter = true;
        HC(iterate_body());
        if (last_solve_status == PFMG_ERR_NAN) return hipSuccess;
    }
    return residual_read(nullptr, block);
}

// Record the launches of fn into an executable graph.  Capture runs on a
// private stream (the caller's stream may be the null stream, which cannot
// be captured); the graph is then launched on the caller's stream.
hipError_t Solver::capture(const std::function<hipError_t()> &fn, hipGraphExec_t *out, long long *vc)
{
    if (!cap) HC(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    // V-cycles are counted on the host as they are enqueued: keep the count
    // of one replay and restore the counters (nothing ran during capture)
    const long long v0 = vcount[0], v1 = vcount[1], v2 = vcount[2];
    hipStream_t saved = s;
    s = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    hipError_t e1 = e == hipSuccess ? fn() : e;
    hipGraph_t g = nullptr;
    hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cap, &g) : e;
    s = saved;
    vc[0] = vcount[0] - v0;
    vc[1] = vcount[1] - v1;
    vc[2] = vcount[2] - v2;
    vcount[0] = v0;
    vcount[1] = v1;
    vcount[2] = v2;
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e1 != hipSuccess ? e1 : e2;
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

void Solver::release_graphs()
{
    if (g_iter) (void)hipGraphExecDestroy(g_iter);
    if (g_start) (void)hipGraphExecDestroy(g_start);
    if (cap) (void)hipStreamDestroy(cap);
    if (s2) (void)hipStreamDestroy(s2);
    if (s3) (void)hipStreamDestroy(s3);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (hipEvent_t &e : evc)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    for (hipEvent_t &e : ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    g_iter = g_start = nullptr;
    cap = s2 = s3 = nullptr;
    ev_fork = nullptr;
}

template hipError_t Solver::smooth<double>(int, int, const int *, double, View<double>, View<double>, View<double>, int, bool);
template hipError_t Solver::smooth<float>(int, int, const int *, double, View<float>, View<float>, View<float>, int, bool);

}  // namespace pfmg
