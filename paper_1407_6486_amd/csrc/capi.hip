// C-ABI entry points declared in include/pfmg.h.  Argument checking,
// status translation and host <-> device staging; the numerical work is in
// solver.hip and the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "batch.h"
#include "solver.h"
#include "tune.h"
#include "unet.h"

struct pfmg_ctx {
    pfmg::Solver sv;
};

struct pfmg_batch {
    pfmg::BatchSolver bs;
};

struct pfmg_nn {
    pfmg::UNet net;
    float *stage = nullptr;   // pinned host copy of the parameters
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
    p->guess_min_relres = 0.0;
    p->stencil_order = 2;
    p->interp_order = 2;
    p->f_solve = 0;
    p->f_interp = 0;
    p->residual_abs = 0;
    p->nodes_middle = 0;
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
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv.hnnsc, sizeof(double) * 2 * sv.P, hipHostMallocDefault);
    // Zero the whole workspace once: halos carry the Dirichlet data.
    if (e == hipSuccess) e = hipMemsetAsync(workspace, 0, need, sv.s);
    if (e == hipSuccess) e = sv.upload_constants();
    if (e != hipSuccess) {
        if (sv.hbits) (void)hipHostFree(sv.hbits);
        if (sv.hmask) (void)hipHostFree(sv.hmask);
        if (sv.hnnsc) (void)hipHostFree(sv.hnnsc);
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
    sv.timer.release();
    if (sv.hbits) (void)hipHostFree(sv.hbits);
    if (sv.hmask) (void)hipHostFree(sv.hmask);
    if (sv.hnnsc) (void)hipHostFree(sv.hnnsc);
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

}  // extern "C"

// ------------------------------------------------- solve without allocation
// Device scratch of pfmg_vcycle_noalloc: one static array per GPU (each
// device that loads the library holds its own copy until the process
// ends).  Host code never passes `scratch` itself to a kernel or copy: the
// name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
namespace pfmg {
namespace noalloc {

__device__ __align__(256) unsigned char scratch[PFMG_NOALLOC_SCRATCH_BYTES];

constexpr int MAXDEV = 64;
std::mutex g_mu;
void *g_ptr[MAXDEV] = {};
// Layout of the last call per device: the scratch is cleared (halo words
// carry the Dirichlet zeros) whenever it changes.
struct Key {
    int dim = 0, n = 0, precision = -1, smoother = -1, stencil_order = 0;
    bool operator==(const Key &o) const
    {
        return dim == o.dim && n == o.n && precision == o.precision && smoother == o.smoother &&
               stencil_order == o.stencil_order;
    }
};
Key g_key[MAXDEV];

// Device address of this device's scratch (nullptr and the error on failure).
hipError_t scratch_ptr(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace noalloc
}  // namespace pfmg

extern "C" {

pfmg_status pfmg_vcycle_noalloc(const pfmg_params *p, double alpha, const double *b, double *u, int32_t n_cycles,
                                void *hip_stream, double *relres_out, int32_t *cycles_out)
{
    namespace na = pfmg::noalloc;
    if (!p || !b || !u) return fail(PFMG_ERR_ARG, "null argument");
    if (!(alpha >= 0) || !std::isfinite(alpha)) return fail(PFMG_ERR_ARG, "alpha must be finite and >= 0");
    if (n_cycles < 0 || n_cycles > 1000) return fail(PFMG_ERR_ARG, "n_cycles must be in 0..1000");
    if (p->guess != PFMG_GUESS_PREV) return fail(PFMG_ERR_ARG, "pfmg_vcycle_noalloc takes guess = PFMG_GUESS_PREV");
    // the fine grid's solve only: one slice, one level
    pfmg_params q = *p;
    q.n_slices = 1;
    q.nodes_coarse = 0;
    q.nodes_middle = 0;
    std::string why;
    if (!pfmg::Solver::validate(q, why)) return fail(PFMG_ERR_ARG, why);
    const size_t need = pfmg::Solver::carve_vcycle(q, nullptr, nullptr);
    if (need > PFMG_NOALLOC_SCRATCH_BYTES)
        return fail(PFMG_ERR_WORKSPACE, "pfmg_vcycle_noalloc: this grid needs " + std::to_string(need) +
                                            " bytes of scratch, the static scratch holds " +
                                            std::to_string((size_t)PFMG_NOALLOC_SCRATCH_BYTES));
    int dev = 0;
    HIPCALL(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= na::MAXDEV) return fail(PFMG_ERR_ARG, "device index beyond the scratch table");
    void *base = nullptr;
    HIPCALL(na::scratch_ptr(dev, &base), "hipGetSymbolAddress(scratch)");
    pfmg::Solver sv;
    sv.p = q;
    sv.s = (hipStream_t)hip_stream;
    if (!sv.init_host(why)) return fail(PFMG_ERR_ARG, why);
    sv.tune = false;
    pfmg::Solver::carve_vcycle(q, (char *)base, &sv);
    // host mirrors of the reduction scratch: pageable, read after a synchronisation
    unsigned long long hbits[4 * pfmg::k::RSLOTS] = {};
    int hmask[1] = {0};
    sv.hbits = hbits;
    sv.hmask = hmask;
    const na::Key key{q.dim, q.n, q.precision, q.smoother, q.stencil_order};
    {
        std::lock_guard<std::mutex> lk(na::g_mu);
        if (!(na::g_key[dev] == key)) {
            HIPCALL(pfmg::k::fill_u64((unsigned long long *)base, 0, (int)(need / 8), sv.s), "clear scratch");
            na::g_key[dev] = key;
        }
    }
    const int n = q.n;
    pfmg::View<double> vb{sv.vb, 0}, vu{sv.vu, 0};
    HIPCALL(pfmg::k::unpack(sv.tl(n, 1), b, vb, sv.s), "unpack b");
    HIPCALL(pfmg::k::unpack(sv.tl(n, 1), u, vu, sv.s), "unpack u");
    double rr = 0;
    HIPCALL(sv.solve(0, vu, vb, 1, alpha, n_cycles, relres_out ? &rr : nullptr), "vcycle");
    const pfmg_status st = sv.last_solve_status;
    HIPCALL(pfmg::k::pack(sv.tl(n, 1), vu, u, sv.s), "pack u");
    if (n_cycles == 0 || relres_out) HIPCALL(hipStreamSynchronize(sv.s), "vcycle");
    if (relres_out) *relres_out = rr;
    if (cycles_out) *cycles_out = (int32_t)sv.vcount[0];
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
    if (field < PFMG_U_FINE || field > PFMG_U_L2_OLD) return fail(PFMG_ERR_ARG, "bad field");
    const int lev = field >= PFMG_U_L2 ? 2 : field >= PFMG_U_COARSE ? 1 : 0;
    if (lev >= sv.nl) return fail(PFMG_ERR_ARG, "no such level");
    const pfmg::PLevel &Lv = sv.L[lev];
    if (slice < 0 || slice >= sv.P || node < 0 || node >= Lv.nn) return fail(PFMG_ERR_ARG, "bad slice or node");
    double *base = nullptr;
    switch (field) {
    case PFMG_U_FINE: case PFMG_U_COARSE: case PFMG_U_L2: base = Lv.U; break;
    case PFMG_F_FINE: case PFMG_F_COARSE: case PFMG_F_L2: base = Lv.F; break;
    case PFMG_TAU: case PFMG_TAU_L2: base = Lv.Tau; break;
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
    if (!ctx || !count_out || level < 0 || level > 2) return fail(PFMG_ERR_ARG, "bad argument");
    *count_out = ctx->sv.vcount[level];
    return PFMG_OK;
}

pfmg_status pfmg_timing_enable(pfmg_ctx *ctx, const char *kernel, int32_t enable)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    HIPCALL(hipStreamSynchronize(ctx->sv.s), "timing");
    if (enable && !kernel) return fail(PFMG_ERR_ARG, "kernel name required");
    HIPCALL(ctx->sv.timer.enable(kernel, enable != 0), "timing events");
    return PFMG_OK;
}

pfmg_status pfmg_timing_read(pfmg_ctx *ctx, int64_t *launches, double *ms_total, double *bytes_total)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    HIPCALL(hipStreamSynchronize(ctx->sv.s), "timing");
    long long nl = 0;
    HIPCALL(ctx->sv.timer.read(&nl, ms_total, bytes_total), "elapsed");
    if (launches) *launches = nl;
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
    bs.timer.release();
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

pfmg_status pfmg_batch_timing_enable(pfmg_batch *b, const char *kernel, int32_t enable)
{
    if (!b) return fail(PFMG_ERR_ARG, "null batch");
    HIPCALL(hipStreamSynchronize(b->bs.s), "timing");
    if (enable && !kernel) return fail(PFMG_ERR_ARG, "kernel name required");
    HIPCALL(b->bs.timer.enable(kernel, enable != 0), "timing events");
    return PFMG_OK;
}

pfmg_status pfmg_batch_timing_read(pfmg_batch *b, int64_t *launches, double *ms_total, double *bytes_total)
{
    if (!b) return fail(PFMG_ERR_ARG, "null batch");
    HIPCALL(hipStreamSynchronize(b->bs.s), "timing");
    long long nl = 0;
    HIPCALL(b->bs.timer.read(&nl, ms_total, bytes_total), "elapsed");
    if (launches) *launches = nl;
    return PFMG_OK;
}

pfmg_status pfmg_batch_vcycle_count(pfmg_batch *b, int32_t level, int64_t *count_out)
{
    if (!b || !count_out || level < 0 || level > 1) return fail(PFMG_ERR_ARG, "bad argument");
    *count_out = b->bs.vcount[level];
    return PFMG_OK;
}

pfmg_status pfmg_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if (bytes == 0) return PFMG_OK;
    if (!dst || !src) return fail(PFMG_ERR_ARG, "null pointer");
    if ((bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return fail(PFMG_ERR_ARG, "bytes and both pointers must be multiples of 16");
    const uintptr_t d = (uintptr_t)dst, sr = (uintptr_t)src;
    if (d < sr + bytes && sr < d + bytes) return fail(PFMG_ERR_ARG, "source and destination overlap");
    HIPCALL(pfmg::k::stream_copy(dst, src, bytes, (hipStream_t)hip_stream), "stream copy");
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

pfmg_status pfmg_tune_set(const char *key, int32_t fused, int32_t ty, int32_t zchunk)
{
    if (!key) return fail(PFMG_ERR_ARG, "null key");
    if (!pfmg::tune_set(key, fused, ty, zchunk)) return fail(PFMG_ERR_ARG, "malformed key or unsupported shape");
    return PFMG_OK;
}

// ---------------------------------------------------------- learned guess
namespace {

// parameters: per layer W [cout][cin][3][3][3] (output layer [1][16][1][1][1])
// then b [cout]; the library keeps W as [27][cout][cin]
void to_kernel_layout(const pfmg::UNet &u, const float *in, float *out)
{
    for (const pfmg::UNetLayer &l : u.L) {
        const int taps = l.kind == 3 ? 1 : 27;
        for (int co = 0; co < l.cout; ++co)
            for (int ci = 0; ci < l.cin; ++ci)
                for (int t = 0; t < taps; ++t)
                    out[l.w_off + ((long)t * l.cout + co) * l.cin + ci] = in[l.w_off + ((long)co * l.cin + ci) * taps + t];
        for (int co = 0; co < l.cout; ++co) out[l.b_off + co] = in[l.b_off + co];
    }
}

void from_kernel_layout(const pfmg::UNet &u, const float *in, float *out)
{
    for (const pfmg::UNetLayer &l : u.L) {
        const int taps = l.kind == 3 ? 1 : 27;
        for (int co = 0; co < l.cout; ++co)
            for (int ci = 0; ci < l.cin; ++ci)
                for (int t = 0; t < taps; ++t)
                    out[l.w_off + ((long)co * l.cin + ci) * taps + t] = in[l.w_off + ((long)t * l.cout + co) * l.cin + ci];
        for (int co = 0; co < l.cout; ++co) out[l.b_off + co] = in[l.b_off + co];
    }
}

uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

}  // namespace

pfmg_status pfmg_nn_param_count(int64_t *count_out)
{
    if (!count_out) return fail(PFMG_ERR_ARG, "null argument");
    *count_out = pfmg::UNet::param_count();
    return PFMG_OK;
}

pfmg_status pfmg_nn_workspace_bytes(int32_t n, int32_t batch, int32_t training, size_t *bytes_out)
{
    if (!bytes_out) return fail(PFMG_ERR_ARG, "null argument");
    if (!pfmg::UNet::valid_n(n)) return fail(PFMG_ERR_ARG, "n must be odd on three levels (n, (n+1)/2-1, ...) >= 3");
    if (batch < 1 || batch > 4096) return fail(PFMG_ERR_ARG, "batch must be in 1..4096");
    pfmg::UNet u;
    u.n[0] = n;
    u.cap = batch;
    u.training = training != 0;
    *bytes_out = u.carve(nullptr);
    return PFMG_OK;
}

pfmg_status pfmg_nn_create(int32_t n, int32_t batch, int32_t training, void *workspace, size_t bytes, void *hip_stream,
                           pfmg_nn **out)
{
    if (!out) return fail(PFMG_ERR_ARG, "null argument");
    *out = nullptr;
    size_t need = 0;
    pfmg_status st = pfmg_nn_workspace_bytes(n, batch, training, &need);
    if (st) return st;
    if (!workspace || bytes < need) return fail(PFMG_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255) != 0) return fail(PFMG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    pfmg_nn *c = new (std::nothrow) pfmg_nn;
    if (!c) return fail(PFMG_ERR_ARG, "out of host memory");
    pfmg::UNet &u = c->net;
    u.n[0] = n;
    u.cap = batch;
    u.training = training != 0;
    u.s = (hipStream_t)hip_stream;
    u.carve((char *)workspace);
    hipError_t e = hipHostMalloc((void **)&c->stage, sizeof(float) * u.nparams, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemsetAsync(workspace, 0, need, u.s);   // halos and moments start at zero
    if (e == hipSuccess) e = hipStreamSynchronize(u.s);
    if (e != hipSuccess) {
        if (c->stage) (void)hipHostFree(c->stage);
        delete c;
        return hip_fail(e, "pfmg_nn_create");
    }
    *out = c;
    return PFMG_OK;
}

pfmg_status pfmg_nn_destroy(pfmg_nn *nn)
{
    if (!nn) return PFMG_OK;
    (void)hipStreamSynchronize(nn->net.s);
    if (nn->stage) (void)hipHostFree(nn->stage);
    delete nn;
    return PFMG_OK;
}

pfmg_status pfmg_nn_load(pfmg_nn *nn, const float *params, int64_t count)
{
    if (!nn || !params) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::UNet &u = nn->net;
    if (count != u.nparams) return fail(PFMG_ERR_ARG, "expected " + std::to_string(u.nparams) + " parameters");
    to_kernel_layout(u, params, nn->stage);
    HIPCALL(hipMemcpyAsync(u.params, nn->stage, sizeof(float) * u.nparams, hipMemcpyHostToDevice, u.s), "nn load");
    HIPCALL(u.refresh_weights(), "nn weights");
    if (u.training) {
        HIPCALL(pfmg::nn::fill_f32(u.m1, 0.f, u.nparams, u.s), "nn moments");
        HIPCALL(pfmg::nn::fill_f32(u.m2, 0.f, u.nparams, u.s), "nn moments");
        u.adam_t = 0;
    }
    HIPCALL(hipStreamSynchronize(u.s), "nn load");
    return PFMG_OK;
}

pfmg_status pfmg_nn_save(pfmg_nn *nn, float *params, int64_t count)
{
    if (!nn || !params) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::UNet &u = nn->net;
    if (count != u.nparams) return fail(PFMG_ERR_ARG, "expected " + std::to_string(u.nparams) + " parameters");
    HIPCALL(hipMemcpyAsync(nn->stage, u.params, sizeof(float) * u.nparams, hipMemcpyDeviceToHost, u.s), "nn save");
    HIPCALL(hipStreamSynchronize(u.s), "nn save");
    from_kernel_layout(u, nn->stage, params);
    return PFMG_OK;
}

pfmg_status pfmg_nn_init(pfmg_nn *nn, uint64_t seed)
{
    if (!nn) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::UNet &u = nn->net;
    std::vector<float> w(u.nparams, 0.f);
    uint64_t st = seed * 0x2545f4914f6cdd1dULL + 1;
    for (const pfmg::UNetLayer &l : u.L) {
        const int taps = l.kind == 3 ? 1 : 27;
        const double sd = std::sqrt(2.0 / (double)(l.cin * taps)) * (l.kind == 3 ? 0.1 : 1.0);
        const long nw = (long)l.cout * l.cin * taps;
        for (long i = 0; i < nw; ++i) {
            // Box-Muller on two uniforms in (0, 1]
            const double u1 = ((splitmix(st) >> 11) + 1.0) * 0x1.0p-53, u2 = (splitmix(st) >> 11) * 0x1.0p-53;
            w[l.w_off + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
    return pfmg_nn_load(nn, w.data(), u.nparams);
}

pfmg_status pfmg_nn_forward(pfmg_nn *nn, const float *x, int32_t batch, float *y)
{
    if (!nn || !x || !y) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::UNet &u = nn->net;
    if (batch < 1 || batch > u.cap) return fail(PFMG_ERR_ARG, "batch exceeds the network's capacity");
    HIPCALL(u.load_dense_input(x, batch), "nn input");
    HIPCALL(u.forward(batch), "nn forward");
    const long n3 = (long)u.n[0] * u.n[0] * u.n[0];
    HIPCALL(hipMemcpyAsync(y, u.y, sizeof(float) * n3 * batch, hipMemcpyDeviceToDevice, u.s), "nn output");
    HIPCALL(hipStreamSynchronize(u.s), "nn forward");
    return PFMG_OK;
}

pfmg_status pfmg_nn_gradients(pfmg_nn *nn, const float *x, const float *target, int32_t batch, double *loss_out,
                              float *grads_out)
{
    if (!nn || !x || !target || !grads_out) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::UNet &u = nn->net;
    if (!u.training) return fail(PFMG_ERR_STATE, "the network was created for inference only");
    if (batch < 1 || batch > u.cap) return fail(PFMG_ERR_ARG, "batch exceeds the network's capacity");
    const long n3 = (long)u.n[0] * u.n[0] * u.n[0];
    HIPCALL(u.load_dense_input(x, batch), "nn input");
    HIPCALL(hipMemcpyAsync(u.target, target, sizeof(float) * n3 * batch, hipMemcpyDeviceToDevice, u.s), "nn target");
    HIPCALL(u.forward(batch), "nn forward");
    HIPCALL(u.backward(batch, (double)n3 * batch), "nn backward");
    double l = 0;
    HIPCALL(hipMemcpyAsync(&l, u.loss, 8, hipMemcpyDeviceToHost, u.s), "nn loss");
    HIPCALL(hipMemcpyAsync(nn->stage, u.grads, sizeof(float) * u.nparams, hipMemcpyDeviceToHost, u.s), "nn grads");
    HIPCALL(hipStreamSynchronize(u.s), "nn gradients");
    from_kernel_layout(u, nn->stage, grads_out);
    if (loss_out) *loss_out = l / ((double)n3 * batch);
    return PFMG_OK;
}

pfmg_status pfmg_nn_train_step(pfmg_nn *nn, const void *pairs, const float *ah2, int32_t n_pairs, const int32_t *idx,
                               int32_t batch, float lr, double *loss_out)
{
    if (!nn || !pairs || !ah2 || !idx) return fail(PFMG_ERR_ARG, "null argument");
    for (int q = 0; q < batch; ++q)
        if (idx[q] < 0 || idx[q] >= n_pairs) return fail(PFMG_ERR_ARG, "pair index out of range");
    pfmg::UNet &u = nn->net;
    if (!u.training) return fail(PFMG_ERR_STATE, "the network was created for inference only");
    if (batch < 1 || batch > u.cap) return fail(PFMG_ERR_ARG, "batch exceeds the network's capacity");
    if (!(lr > 0)) return fail(PFMG_ERR_ARG, "lr must be positive");
    HIPCALL(u.train_step((const pfmg::nn::bf16 *)pairs, ah2, idx, batch, lr, loss_out), "nn train step");
    return PFMG_OK;
}

pfmg_status pfmg_nn_tensor(pfmg_nn *nn, int32_t layer, int32_t which, int32_t batch, float *dst)
{
    if (!nn || !dst) return fail(PFMG_ERR_ARG, "null argument");
    pfmg::UNet &u = nn->net;
    if (layer < 0 || layer > 12 || which < 0 || which > 3) return fail(PFMG_ERR_ARG, "layer in 0..12, which in 0..3");
    if (batch < 1 || batch > u.cap) return fail(PFMG_ERR_ARG, "bad batch");
    if (which >= 2 && !u.training) return fail(PFMG_ERR_STATE, "gradients need a training network");
    if (which == 3 && layer == 0) return fail(PFMG_ERR_ARG, "the first layer has no input gradient");
    const pfmg::UNetLayer &l = u.L[layer];
    const pfmg::nn::Act a = which == 0 ? l.in : which == 1 ? l.out : which == 2 ? l.dout : l.din;
    const int c = (which == 0 || which == 3) ? l.cin : l.cout;
    HIPCALL(pfmg::nn::act_to_dense(a, c, batch, dst, u.s), "nn tensor");
    HIPCALL(hipStreamSynchronize(u.s), "nn tensor");
    return PFMG_OK;
}

pfmg_status pfmg_attach_nn(pfmg_ctx *ctx, pfmg_nn *nn)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    pfmg::Solver &sv = ctx->sv;
    if (nn) {
        if (sv.p.guess != PFMG_GUESS_LEARNED) return fail(PFMG_ERR_ARG, "the context was created with guess = PFMG_GUESS_PREV");
        if (nn->net.n[0] != sv.p.n) return fail(PFMG_ERR_ARG, "network grid differs from the context's fine grid");
        if (nn->net.cap < sv.P) return fail(PFMG_ERR_ARG, "network batch must hold every slice");
    }
    sv.unet = nn ? &nn->net : nullptr;
    return PFMG_OK;
}

pfmg_status pfmg_guess_stats(pfmg_ctx *ctx, int64_t *tried, int64_t *taken)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    if (tried) *tried = ctx->sv.guess_tried;
    if (taken) *taken = ctx->sv.guess_taken;
    return PFMG_OK;
}

pfmg_status pfmg_record(pfmg_ctx *ctx, void *pairs, float *ah2, double *scratch, int32_t capacity)
{
    if (!ctx) return fail(PFMG_ERR_ARG, "null context");
    pfmg::Solver &sv = ctx->sv;
    if (pairs && (!ah2 || !scratch || capacity < sv.P)) return fail(PFMG_ERR_ARG, "recording needs pairs, ah2, scratch and capacity >= P");
    if (pairs && (sv.p.dim != 3 || sv.p.vcycles_per_solve != 0))
        return fail(PFMG_ERR_ARG, "recording takes the full node solves of a 3D context (vcycles_per_solve = 0)");
    sv.rec_pairs = (__bf16 *)pairs;
    sv.rec_ah2 = ah2;
    sv.rec_scratch = scratch;
    sv.rec_cap = pairs ? capacity : 0;
    sv.rec_count = 0;
    return PFMG_OK;
}

pfmg_status pfmg_record_count(pfmg_ctx *ctx, int32_t *count_out)
{
    if (!ctx || !count_out) return fail(PFMG_ERR_ARG, "null argument");
    *count_out = ctx->sv.rec_count;
    return PFMG_OK;
}

}  // extern "C"
