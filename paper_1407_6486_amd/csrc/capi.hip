// C-ABI entry points declared in include/pfmg.h.  Argument checking,
// status translation and host <-> device staging; the numerical work is in
// solver.hip and the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "batch.h"
#include "solver.h"
#include "tune.h"

struct pfmg_ctx {
    pfmg::Solver sv;
};

struct pfmg_batch {
    pfmg::BatchSolver bs;
};

namespace {

thread_local std::string g_err;

pfmg_status fail(pfmg_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

pfmg_status hip_fail(hipError_t e, const char *where)
{
    return fail(PFMG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCALL(x, where)                                  \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return hip_fail(e_, where);  \
    } while (0)

pfmg_status solve_status(pfmg::Solver &sv)
{
    if (sv.last_solve_status == PFMG_ERR_NAN) return fail(PFMG_ERR_NAN, "a norm evaluated to NaN or Inf");
    return PFMG_OK;
}

}  // namespace

extern "C" {

const char *pfmg_last_error(void) { return g_err.c_str(); }

pfmg_status pfmg_default_params(pfmg_params *p)
{
    if (!p) return fail(PFMG_ERR_ARG, "null params");
    std::memset(p, 0, sizeof *p);
    p->dim = 3;
    p->n = 127;
    p->nu = 1.0;
    p->dt = 1e-3;
    p->n_slices = 16;
    p->nodes_fine = 5;
    p->nodes_coarse = 3;
    p->node_family = PFMG_NODES_LOBATTO;
    p->smoother = PFMG_SMOOTH_RBGS;
    p->nu_pre = 2;
    p->nu_post = 2;
    p->omega = 1.0;
    p->vcycles_per_solve = 1;
    p->mg_tol = 1e-12;
    p->mg_stall = 0.75;
    p->mg_max_cycles = 50;
    p->precision = PFMG_FP64;
    p->guess = PFMG_GUESS_PREV;
    p->fine_send = PFMG_SEND_AFTER_ITER;
    p->pfasst_tol = 1e-10;
    p->pfasst_max_iter = 200;
    return PFMG_OK;
}

pfmg_status pfmg_workspace_bytes(const pfmg_params *p, size_t *bytes_out)
{
    if (!p || !bytes_out) return fail(PFMG_ERR_ARG, "null argument");
    std::string why;
    if (!pfmg::Solver::validate(*p, why)) return fail(PFMG_ERR_ARG, why);
    *bytes_out = pfmg::Solver::carve(*p, nullptr, nullptr);
    return PFMG_OK;
}

pfmg_status pfmg_create(const pfmg_params *p, void *workspace, size_t bytes, void *hip_stream, pfmg_ctx **out)
{
    if (!p || !out) return fail(PFMG_ERR_ARG, "null argument");
    *out = nullptr;
    std::string why;
    if (!pfmg::Solver::validate(*p, why)) return fail(PFMG_ERR_ARG, why);
    const size_t need = pfmg::Solver::carve(*p, nullptr, nullptr);
    if (!workspace || bytes < need)
        return fail(PFMG_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255) != 0) return fail(PFMG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    pfmg_ctx *c = new (std::nothrow) pfmg_ctx;
    if (!c) return fail(PFMG_ERR_ARG, "out of host memory");
    pfmg::Solver &sv = c->sv;
    sv.p = *p;
    sv.s = (hipStream_t)hip_stream;
    if (!sv.init_host(why)) { delete c; return fail(PFMG_ERR_ARG, why); }
    pfmg::Solver::carve(*p, (char *)workspace, &sv);
    hipError_t e = hipHostMalloc((void **)&sv.hbits, sizeof(unsigned long long) * 4 * sv.P * pfmg::k::RSLOTS, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv.hmask, sizeof(int) * sv.P, hipHostMallocDefault);
    // Zero the whole workspace once: halos carry the Dirichlet data.
    if (e == hipSuccess) e = hipMemsetAsync(workspace, 0, need, sv.s);
    if (e == hipSuccess) e = sv.upload_constants();
    if (e != hipSuccess) {
        if (sv.hbits) (void)hipHostFree(sv.hbits);
        if (sv.hmask) (void)hipHostFree(sv.hmask);
        delete c;
        return hip_fail(e, "pfmg_create");
    }
    *out = c;
    return PFMG_OK;
}

pfmg_status pfmg_destroy(pfmg_ctx *ctx)
{
    if (!ctx) return PFMG_OK;
    pfmg::Solver &sv = ctx->sv;
    (void)hipStreamSynchronize(sv.s);
    sv.release_graphs();
    for (hipEvent_t ev : sv.timer.ev) (void)hipEventDestroy(ev);
    if (sv.hbits) (void)hipHostFree(sv.hbits);
    if (sv.hmask) (void)hipHostFree(sv.hmask);
    delete ctx;
    return PFMG_OK;
}

pfmg_status pfmg_set_initial(pfmg_ctx *ctx, const double *u0, int32_t on_device)
{
    if (!ctx || !u0) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::Solver &sv = ctx->sv;
    const long pts = pfmg::interior_points(sv.p.n, sv.dim);
    const double *src = u0;
    if (!on_device) {
        HIPCALL(hipMemcpyAsync(sv.vb, u0, sizeof(double) * pts, hipMemcpyHostToDevice, sv.s), "copy u0");
        src = sv.vb;
    }
    HIPCALL(sv.spread(src), "spread and predictor");
    HIPCALL(hipStreamSynchronize(sv.s), "set_initial");
    sv.has_state = true;
    return solve_status(sv);
}

pfmg_status pfmg_sdc_sweep(pfmg_ctx *ctx, int32_t level, int32_t p_begin, int32_t p_end)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    pfmg::Solver &sv = ctx->sv;
    if (level < 0 || level >= sv.nl) return fail(PFMG_ERR_ARG, "no such level");
    if (p_begin < 0 || p_end > sv.P || p_begin > p_end) return fail(PFMG_ERR_ARG, "bad slice range");
    if (!sv.has_state) return fail(PFMG_ERR_STATE, "set_initial first");
    HIPCALL(sv.sweep(level, p_begin, p_end), "sweep");
    HIPCALL(hipStreamSynchronize(sv.s), "sweep");
    return solve_status(sv);
}

pfmg_status pfmg_vcycle(pfmg_ctx *ctx, double alpha, const double *b, double *u, int32_t n_cycles,
                        double *relres_out, int32_t *cycles_out)
{
    if (!ctx || !b || !u) return fail(PFMG_ERR_ARG, "null argument");
    if (!(alpha >= 0) || !std::isfinite(alpha)) return fail(PFMG_ERR_ARG, "alpha must be finite and >= 0");
    if (n_cycles < 0 || n_cycles > 1000) return fail(PFMG_ERR_ARG, "n_cycles must be in 0..1000");
    pfmg::Solver &sv = ctx->sv;
    const int n = sv.p.n;
    pfmg::View<double> vb{sv.vb, 0}, vu{sv.vu, 0};
    HIPCALL(pfmg::k::unpack(sv.tl(n, 1), b, vb, sv.s), "unpack b");
    HIPCALL(pfmg::k::unpack(sv.tl(n, 1), u, vu, sv.s), "unpack u");
    const long long before = sv.vcount[0];
    double rr = 0;
    HIPCALL(sv.solve(0, vu, vb, 1, alpha, n_cycles, &rr), "vcycle");
    const pfmg_status st = sv.last_solve_status;
    HIPCALL(pfmg::k::pack(sv.tl(n, 1), vu, u, sv.s), "pack u");
    HIPCALL(hipStreamSynchronize(sv.s), "vcycle");
    if (relres_out) *relres_out = rr;
    if (cycles_out) *cycles_out = (int32_t)(sv.vcount[0] - before);
    sv.vcount[0] = before;
    if (st == PFMG_ERR_NAN) return fail(PFMG_ERR_NAN, "a norm evaluated to NaN or Inf");
    return st;
}

pfmg_status pfmg_pfasst_iter(pfmg_ctx *ctx, double *block_res_out)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    pfmg::Solver &sv = ctx->sv;
    if (!sv.has_state) return fail(PFMG_ERR_STATE, "set_initial first");
    double blk = 0;
    HIPCALL(sv.iterate(&blk), "iteration");
    if (block_res_out) *block_res_out = blk;
    return solve_status(sv);
}

pfmg_status pfmg_residual(pfmg_ctx *ctx, int32_t level, double *per_slice_out)
{
    if (!ctx || !per_slice_out) return fail(PFMG_ERR_ARG, "null argument");
    if (level != 0) return fail(PFMG_ERR_ARG, "the residual is defined on level 0");
    pfmg::Solver &sv = ctx->sv;
    if (!sv.has_state) return fail(PFMG_ERR_STATE, "set_initial first");
    HIPCALL(sv.residual(per_slice_out, nullptr), "residual");
    return solve_status(sv);
}

pfmg_status pfmg_run_block(pfmg_ctx *ctx, const double *u0, int32_t on_device, int32_t *iters_out, double *res_out)
{
    pfmg_status st = pfmg_set_initial(ctx, u0, on_device);
    if (st < 0) return st;
    pfmg::Solver &sv = ctx->sv;
    double blk = INFINITY;
    int it = 0;
    while (it < sv.p.pfasst_max_iter) {
        st = pfmg_pfasst_iter(ctx, &blk);
        ++it;
        if (st < 0) return st;
        if (blk <= sv.p.pfasst_tol) break;
    }
    if (iters_out) *iters_out = it;
    if (res_out) *res_out = blk;
    return blk <= sv.p.pfasst_tol ? PFMG_OK : PFMG_NOT_CONVERGED;
}

static pfmg_status field_ptr(pfmg::Solver &sv, int32_t field, int32_t slice, int32_t node, double **out, int *n)
{
    const bool coarse = field >= PFMG_U_COARSE;
    if (field < PFMG_U_FINE || field > PFMG_U_COARSE_OLD) return fail(PFMG_ERR_ARG, "bad field");
    if (coarse && sv.nl < 2) return fail(PFMG_ERR_ARG, "no coarse level");
    const pfmg::PLevel &Lv = sv.L[coarse ? 1 : 0];
    if (slice < 0 || slice >= sv.P || node < 0 || node >= Lv.nn) return fail(PFMG_ERR_ARG, "bad slice or node");
    double *base = nullptr;
    switch (field) {
    case PFMG_U_FINE: case PFMG_U_COARSE: base = Lv.U; break;
    case PFMG_F_FINE: case PFMG_F_COARSE: base = Lv.F; break;
    case PFMG_TAU: base = Lv.Tau; break;
    default: base = Lv.Uold; break;
    }
    *out = Lv.slot(base, slice, node);
    *n = Lv.n;
    return PFMG_OK;
}

pfmg_status pfmg_get(pfmg_ctx *ctx, int32_t field, int32_t slice, int32_t node, double *dst, int32_t on_device)
{
    if (!ctx || !dst) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::Solver &sv = ctx->sv;
    double *f;
    int n;
    pfmg_status st = field_ptr(sv, field, slice, node, &f, &n);
    if (st) return st;
    const long pts = pfmg::interior_points(n, sv.dim);
    double *target = on_device ? dst : sv.vb;
    HIPCALL(pfmg::k::pack(sv.tl(n, 1), pfmg::View<double>{f, 0}, target, sv.s), "pack");
    if (!on_device) HIPCALL(hipMemcpyAsync(dst, sv.vb, sizeof(double) * pts, hipMemcpyDeviceToHost, sv.s), "copy");
    HIPCALL(hipStreamSynchronize(sv.s), "get");
    return PFMG_OK;
}

pfmg_status pfmg_set(pfmg_ctx *ctx, int32_t field, int32_t slice, int32_t node, const double *src, int32_t on_device)
{
    if (!ctx || !src) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::Solver &sv = ctx->sv;
    double *f;
    int n;
    pfmg_status st = field_ptr(sv, field, slice, node, &f, &n);
    if (st) return st;
    const long pts = pfmg::interior_points(n, sv.dim);
    const double *from = src;
    if (!on_device) {
        HIPCALL(hipMemcpyAsync(sv.vb, src, sizeof(double) * pts, hipMemcpyHostToDevice, sv.s), "copy");
        from = sv.vb;
    }
    HIPCALL(pfmg::k::unpack(sv.tl(n, 1), from, pfmg::View<double>{f, 0}, sv.s), "unpack");
    HIPCALL(hipStreamSynchronize(sv.s), "set");
    sv.has_state = true;
    return PFMG_OK;
}

pfmg_status pfmg_vcycle_count(pfmg_ctx *ctx, int32_t level, int64_t *count_out)
{
    if (!ctx || !count_out || level < 0 || level > 1) return fail(PFMG_ERR_ARG, "bad argument");
    *count_out = ctx->sv.vcount[level];
    return PFMG_OK;
}

pfmg_status pfmg_timing_enable(pfmg_ctx *ctx, const char *kernel, int32_t enable)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    pfmg::Timer &t = ctx->sv.timer;
    HIPCALL(hipStreamSynchronize(ctx->sv.s), "timing");
    t.on = enable != 0;
    t.used = 0;
    t.depth = 0;
    t.open = -1;
    t.bytes = 0;
    t.launches = 0;
    if (!t.on) return PFMG_OK;
    if (!kernel) return fail(PFMG_ERR_ARG, "kernel name required");
    t.key = kernel;
    if (t.ev.empty()) {
        t.ev.resize(1 << 16);
        for (auto &ev : t.ev) HIPCALL(hipEventCreate(&ev), "event");
    }
    return PFMG_OK;
}

pfmg_status pfmg_timing_read(pfmg_ctx *ctx, int64_t *launches, double *ms_total, double *bytes_total)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    pfmg::Timer &t = ctx->sv.timer;
    HIPCALL(hipStreamSynchronize(ctx->sv.s), "timing");
    double ms = 0;
    for (size_t q = 0; q + 1 < t.used; q += 2) {
        float e = 0;
        HIPCALL(hipEventElapsedTime(&e, t.ev[q], t.ev[q + 1]), "elapsed");
        ms += e;
    }
    if (launches) *launches = t.launches;
    if (ms_total) *ms_total = ms;
    if (bytes_total) *bytes_total = t.bytes;
    return PFMG_OK;
}

// ------------------------------------------------------------------ batch
pfmg_status pfmg_batch_workspace_bytes(const pfmg_params *pp, int32_t np, size_t *bytes_out)
{
    if (!pp || !bytes_out) return fail(PFMG_ERR_ARG, "null argument");
    std::string why;
    if (!pfmg::BatchSolver::validate(pp, np, why)) return fail(PFMG_ERR_ARG, why);
    pfmg::BatchSolver tmp;
    if (!tmp.init_host(pp, np, why)) return fail(PFMG_ERR_ARG, why);
    *bytes_out = tmp.carve(nullptr);
    return PFMG_OK;
}

pfmg_status pfmg_batch_create(const pfmg_params *pp, int32_t np, void *workspace, size_t bytes, void *hip_stream,
                              pfmg_batch **out)
{
    if (!pp || !out) return fail(PFMG_ERR_ARG, "null argument");
    *out = nullptr;
    std::string why;
    if (!pfmg::BatchSolver::validate(pp, np, why)) return fail(PFMG_ERR_ARG, why);
    pfmg_batch *c = new (std::nothrow) pfmg_batch;
    if (!c) return fail(PFMG_ERR_ARG, "out of host memory");
    pfmg::BatchSolver &bs = c->bs;
    if (!bs.init_host(pp, np, why)) { delete c; return fail(PFMG_ERR_ARG, why); }
    const size_t need = bs.carve(nullptr);
    if (!workspace || bytes < need) {
        delete c;
        return fail(PFMG_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    }
    if (((uintptr_t)workspace & 255) != 0) { delete c; return fail(PFMG_ERR_WORKSPACE, "workspace must be 256-byte aligned"); }
    bs.s = (hipStream_t)hip_stream;
    bs.carve((char *)workspace);
    const size_t nb = (size_t)2 * bs.total_items * pfmg::k::RSLOTS;
    hipError_t e = hipHostMalloc((void **)&bs.hbits, sizeof(unsigned long long) * nb, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&bs.hact, sizeof(int) * bs.act_init.size(), hipHostMallocDefault);
    // zero the whole workspace once: halos carry the Dirichlet data
    if (e == hipSuccess) e = hipMemsetAsync(workspace, 0, need, bs.s);
    if (e == hipSuccess) e = bs.upload();
    if (e != hipSuccess) {
        if (bs.hbits) (void)hipHostFree(bs.hbits);
        if (bs.hact) (void)hipHostFree(bs.hact);
        delete c;
        return hip_fail(e, "pfmg_batch_create");
    }
    *out = c;
    return PFMG_OK;
}

pfmg_status pfmg_batch_destroy(pfmg_batch *b)
{
    if (!b) return PFMG_OK;
    pfmg::BatchSolver &bs = b->bs;
    (void)hipStreamSynchronize(bs.s);
    bs.release();
    if (bs.hbits) (void)hipHostFree(bs.hbits);
    if (bs.hact) (void)hipHostFree(bs.hact);
    delete b;
    return PFMG_OK;
}

pfmg_status pfmg_batch_set_initial(pfmg_batch *b, const double *u0, int32_t on_device)
{
    if (!b || !u0) return fail(PFMG_ERR_ARG, "null argument");
    HIPCALL(b->bs.set_initial(u0, on_device != 0), "batch set_initial");
    return PFMG_OK;
}

pfmg_status pfmg_batch_pfasst_iter(pfmg_batch *b, double *res_out)
{
    if (!b) return fail(PFMG_ERR_ARG, "null batch");
    pfmg::BatchSolver &bs = b->bs;
    if (!bs.has_state) return fail(PFMG_ERR_STATE, "set_initial first");
    HIPCALL(bs.iterate(), "batch iteration");
    if (res_out) std::memcpy(res_out, bs.res.data(), sizeof(double) * bs.NP);
    if (bs.nan) return fail(PFMG_ERR_NAN, "a residual evaluated to NaN or Inf");
    return PFMG_OK;
}

pfmg_status pfmg_batch_run(pfmg_batch *b, const double *u0, int32_t on_device, int32_t *iters_out, double *res_out)
{
    pfmg_status st = pfmg_batch_set_initial(b, u0, on_device);
    if (st < 0) return st;
    pfmg::BatchSolver &bs = b->bs;
    for (int it = 0; it < bs.p.pfasst_max_iter; ++it) {
        bool any = false;
        for (char a : bs.active) any = any || a;
        if (!any) break;
        st = pfmg_batch_pfasst_iter(b, nullptr);
        if (st < 0) return st;
    }
    bool all = true;
    for (int q = 0; q < bs.NP; ++q) {
        if (iters_out) iters_out[q] = bs.iters[q];
        if (res_out) res_out[q] = bs.res[q];
        all = all && !bs.active[q];
    }
    return all ? PFMG_OK : PFMG_NOT_CONVERGED;
}

pfmg_status pfmg_batch_get(pfmg_batch *b, int32_t problem, int32_t field, int32_t slice, int32_t node, double *dst,
                           int32_t on_device)
{
    if (!b || !dst) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::BatchSolver &bs = b->bs;
    if (problem < 0 || problem >= bs.NP) return fail(PFMG_ERR_ARG, "bad problem");
    if (field < PFMG_U_FINE || field > PFMG_U_COARSE_OLD) return fail(PFMG_ERR_ARG, "bad field");
    const bool coarse = field >= PFMG_U_COARSE;
    if (coarse && bs.nl < 2) return fail(PFMG_ERR_ARG, "no coarse level");
    if (slice < 0 || slice >= bs.P || node < 0 || node >= bs.nn[coarse ? 1 : 0])
        return fail(PFMG_ERR_ARG, "bad slice or node");
    HIPCALL(bs.get(problem, field, slice, node, dst, on_device != 0), "batch get");
    return PFMG_OK;
}

pfmg_status pfmg_batch_vcycle_count(pfmg_batch *b, int32_t level, int64_t *count_out)
{
    if (!b || !count_out || level < 0 || level > 1) return fail(PFMG_ERR_ARG, "bad argument");
    *count_out = b->bs.vcount[level];
    return PFMG_OK;
}

pfmg_status pfmg_tune_count(int32_t *count_out)
{
    if (!count_out) return fail(PFMG_ERR_ARG, "null argument");
    *count_out = pfmg::tune_table_size();
    return PFMG_OK;
}

pfmg_status pfmg_tune_lookup(const char *key, char *buf, size_t len)
{
    if (!key || !buf || len == 0) return fail(PFMG_ERR_ARG, "null argument");
    const std::string v = pfmg::tune_lookup(key);
    std::snprintf(buf, len, "%s", v.c_str());
    return PFMG_OK;
}

}  // extern "C"
