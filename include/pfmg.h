/*
 * pfmg — IPFASST (PFASST with inexact multigrid node solves) for the heat
 * equation u_t = nu * Laplace(u) on the unit interval or cube with
 * homogeneous Dirichlet data, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Minion, Speck, Bolten, Emmett, Ruprecht, "Interweaving PFASST and
 * Parallel Multigrid", arXiv:1407.6486.
 *   - collocation problem per time slice: eq. collocation / bigPmatk_2 (Sec. 2.1)
 *   - SDC sweep with backward-Euler substeps: eq. sdc-be, SDCcompactLIII (Sec. 2.2)
 *   - collocation residual: eq. resid (Sec. 2.2.2)
 *   - two-level MLSDC with the FAS correction (Sec. 2.3), IMLSDC (Sec. 2.3.1)
 *   - PFASST / IPFASST: predictor, iteration, send-forward (Sec. 2.4, 2.4.1)
 *   - node solves by geometric multigrid V-cycles: linear interpolation,
 *     full-weighting restriction, pre/post smoothing (Sec. 4.1.1, 4.2.1)
 *   - spatial operator: 2nd-order finite differences (3-point in 1D, Sec. 4.1;
 *     7-point in 3D, Sec. 4.2)
 *
 * Conventions for every entry point
 *   - All functions return a pfmg_status.  No C++ exception crosses the ABI.
 *     On an error status (< 0) pfmg_last_error() returns a thread-local
 *     message; the context stays usable except after PFMG_ERR_HIP.
 *   - Work is enqueued on the HIP stream given to pfmg_create.  Calls that
 *     return host scalars (residuals, norms) synchronise that stream.
 *   - Host and device arrays exchanged with the library are dense float64
 *     arrays of n^dim interior values in C order with x fastest; the halo
 *     and padding of the internal layout are never visible to callers.
 *   - Input pointers are borrowed for the duration of the call only.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef PFMG_H
#define PFMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfmg_ctx pfmg_ctx;
typedef int32_t pfmg_status;

enum {
    PFMG_OK = 0,
    PFMG_NOT_CONVERGED = 1,   /* warning: outputs valid, tolerance not met   */
    PFMG_STALLED = 2,         /* warning: MG stall criterion stopped a solve */
    PFMG_ERR_ARG = -1,        /* invalid argument or parameter combination   */
    PFMG_ERR_WORKSPACE = -2,  /* workspace missing, too small or misaligned  */
    PFMG_ERR_HIP = -3,        /* a HIP runtime call failed                   */
    PFMG_ERR_STATE = -4,      /* call out of order (e.g. iterate before set) */
    PFMG_ERR_NAN = -5         /* a norm evaluated to NaN or Inf              */
};

enum { PFMG_NODES_LOBATTO = 0, PFMG_NODES_UNIFORM = 1 };
enum { PFMG_SMOOTH_JACOBI = 0, PFMG_SMOOTH_RBGS = 1 };
enum { PFMG_FP64 = 0, PFMG_MIXED = 1 };
enum { PFMG_GUESS_PREV = 0, PFMG_GUESS_LEARNED = 1 };
enum { PFMG_SEND_AFTER_ITER = 0, PFMG_SEND_AFTER_SWEEP = 1 };
/* Fields readable / writable with pfmg_get / pfmg_set. */
enum { PFMG_U_FINE = 0, PFMG_F_FINE = 1, PFMG_U_COARSE = 2, PFMG_F_COARSE = 3,
       PFMG_TAU = 4, PFMG_U_COARSE_OLD = 5,
       /* level 2 of a three-level context (fields 2..5 are its level 1) */
       PFMG_U_L2 = 6, PFMG_F_L2 = 7, PFMG_TAU_L2 = 8, PFMG_U_L2_OLD = 9 };

/*
 * Problem and method parameters.
 *   dim              1 or 3.
 *   n                interior points per dimension of the fine grid; mesh
 *                    width h = 1/(n+1).  Every multigrid level with n >= 3
 *                    must be odd: the hierarchy n -> (n+1)/2 - 1 ends at
 *                    n in {1, 2}, which is solved exactly.
 *   nu, dt           diffusion coefficient (> 0) and slice length (> 0).
 *   n_slices         P, the time slices of one PFASST block (>= 1).
 *   nodes_fine       nodes per slice on the fine level (2..9), the left end
 *                    point included.
 *   nodes_coarse     nodes on the coarse PFASST level (a subset of the fine
 *                    nodes: 3 with 5 fine nodes, 2 with 3), or 0 for a
 *                    single level (ISDC).  The coarse level uses the grid
 *                    (n+1)/2 - 1.
 *   node_family      PFMG_NODES_LOBATTO: Gauss-Lobatto nodes, the quadrature
 *                    through every node (Sec. 2.1).  PFMG_NODES_UNIFORM:
 *                    nodes m/M (M = nodes - 1) with a quadrature that leaves
 *                    out the left end point (q_{m,0} = 0, f interpolated
 *                    through nodes 1..M), the paper's second-order (3 nodes)
 *                    and fourth-order (5 nodes) methods of Sec. 3 and 4.3;
 *                    2 nodes give backward Euler.
 *   smoother         PFMG_SMOOTH_JACOBI (weighted, omega) or
 *                    PFMG_SMOOTH_RBGS (red = (i+j+k) even in 1-based
 *                    interior indices, red then black, weight omega).
 *   nu_pre, nu_post  smoothing sweeps before / after the coarse correction.
 *   vcycles_per_solve  > 0: exactly that many V-cycles per node solve (the
 *                    inexact solves of IMLSDC/IPFASST); 0: full solve, cycles
 *                    repeat while |b - H u|_inf > mg_tol |b|_inf and each
 *                    cycle cuts the residual below mg_stall times the
 *                    previous one, at most mg_max_cycles (Sec. 4.2.1).
 *   precision        PFMG_FP64, or PFMG_MIXED: FP32 smoothing, restriction,
 *                    prolongation and coarsest solve inside FP64 iterative
 *                    refinement (FP64 residual, FP64 update; one refinement
 *                    step per V-cycle of the solve policy).
 *   guess            PFMG_GUESS_PREV (previous iterate at the same node), or
 *                    PFMG_GUESS_LEARNED (the judged network guess below; 3D
 *                    full solves only).
 *   fine_send        PFMG_SEND_AFTER_ITER: slice p takes slice p-1's end
 *                    value after p-1's previous iteration (after its coarse
 *                    correction).  PFMG_SEND_AFTER_SWEEP (Sec. 2.4: a level
 *                    sends after its sweep): slice p takes slice p-1's end
 *                    value right after p-1's fine sweep of the previous
 *                    iteration (the predictor's end value before the first
 *                    iteration); costs one fine field per slice of
 *                    workspace.  Single contexts only (batches take
 *                    AFTER_ITER).
 *   pfasst_tol       block relative residual tolerance for pfmg_run_block.
 *   pfasst_max_iter  iteration cap for pfmg_run_block.
 *   guess_min_relres with PFMG_GUESS_LEARNED: a node solve is offered the
 *                    network's guess only while its plain guess has
 *                    |b - H U|_inf > guess_min_relres |b|_inf (0: always).
 *   stencil_order    2, or 4: the fine level's Laplacian is fourth order
 *                    (per axis (-u_{i-2} + 16u_{i-1} - 30u_i + 16u_{i+1}
 *                    - u_{i+2}) / 12h^2, the value two steps beyond the
 *                    boundary the odd reflection of the interior one) as in
 *                    the fourth-order runs of Sec. 4.3.  F, the node solves
 *                    (a V-cycle whose finest level smooths with L4 --
 *                    weighted Jacobi, or red-black JOR with each colour from
 *                    the values before its pass -- above the second-order
 *                    cycle) and the residual use it; the coarse PFASST level
 *                    stays second order.  FP64, plain guesses, single
 *                    contexts only.
 *   interp_order     PFASST spatial interpolation of the coarse correction:
 *                    2 d-linear, 4 tensor-product cubic (Sec. 4.3; needs a
 *                    coarse grid of n >= 3).  Single contexts only.
 *   f_solve          F at a node after its implicit-Euler solve (both
 *                    levels): 0 nu L_h U; 1 (U - b) / (dt d_m), the value
 *                    the substep implies (equal to nu L_h U when the solve
 *                    is exact; Sec. 2.2 leaves the choice open).  F at
 *                    node 0 is nu L_h of its value either way.
 *   f_interp         after the coarse correction: 0 the fine F values are
 *                    re-evaluated on the corrected U; 1 they take the coarse
 *                    F change interpolated like U's (time and space).  With
 *                    either option the stored F differs from F(U) until the
 *                    iteration converges, so the collocation residual
 *                    (pfmg_residual, the block residual) evaluates F(U)
 *                    itself.  Single contexts only; both default to 0.
 *   residual_abs     0: each slice's collocation residual is relative to
 *                    its initial value's max-norm (the default); 1: the
 *                    plain max-norm, for an absolute pfasst_tol.  Single
 *                    contexts only.
 *   nodes_middle     0: one or two PFASST levels; > 0 (with nodes_coarse >
 *                    0): three levels, fine (n, nodes_fine), middle
 *                    ((n+1)/2 - 1, nodes_middle) and coarse (one more
 *                    halving, nodes_coarse), each level's nodes a subset of
 *                    the finer one's (Sec. 4.2's weak-scaling runs).  The
 *                    FAS term of the coarse level carries the middle
 *                    level's through the restriction; an iteration sweeps
 *                    the middle level after the restriction and again after
 *                    the coarse correction; the predictor interpolates
 *                    straight up.  Single contexts only; the iteration runs
 *                    the slices in one group (no pipelined schedule).
 */
typedef struct pfmg_params {
    int32_t dim;
    int32_t n;
    double nu;
    double dt;
    int32_t n_slices;
    int32_t nodes_fine;
    int32_t nodes_coarse;
    int32_t node_family;
    int32_t smoother;
    int32_t nu_pre;
    int32_t nu_post;
    double omega;
    int32_t vcycles_per_solve;
    double mg_tol;
    double mg_stall;
    int32_t mg_max_cycles;
    int32_t precision;
    int32_t guess;
    int32_t fine_send;
    double pfasst_tol;
    int32_t pfasst_max_iter;
    double guess_min_relres;
    int32_t stencil_order;
    int32_t interp_order;
    int32_t f_solve;
    int32_t f_interp;
    int32_t residual_abs;
    int32_t nodes_middle;
} pfmg_params;

/* Fills *p with the defaults: 3D, n = 127, nu = 1, dt = 1e-3, 16 slices,
 * 5/3 Lobatto nodes, red-black Gauss-Seidel V(2,2), omega 1, one V-cycle per
 * solve, mg_tol 1e-12, stall 0.75, 50 cycles, FP64, pfasst_tol 1e-10,
 * 200 iterations. */
pfmg_status pfmg_default_params(pfmg_params *p);

/* Device bytes the context needs for these parameters (>= 256-byte aligned
 * workspace).  Errors: PFMG_ERR_ARG for invalid parameters. */
pfmg_status pfmg_workspace_bytes(const pfmg_params *p, size_t *bytes_out);

/* Create a context.  `workspace` is caller-owned device memory of at least
 * pfmg_workspace_bytes (256-byte aligned); it must outlive the context and
 * is not freed by the library.  `hip_stream` is a hipStream_t (NULL = the
 * default stream).  The library allocates no device memory itself; it keeps
 * one small pinned host buffer for residual read-back.  Computes the
 * collocation matrices (Sec. 2.1, eq. Qbe) on the host in long double. */
pfmg_status pfmg_create(const pfmg_params *p, void *workspace, size_t bytes,
                        void *hip_stream, pfmg_ctx **out);
pfmg_status pfmg_destroy(pfmg_ctx *ctx);
/* Message of the last error on this thread ("" if none). */
const char *pfmg_last_error(void);

/* Start a block: copy u0 (n^dim float64, host if on_device == 0, device
 * otherwise) to every node of every slice, evaluate F = nu L u, and — with
 * two levels — run the PFASST predictor (Sec. 2.4: FAS restriction of
 * the spread state, P pipelined rounds of coarse sweeps in which slice p
 * sweeps p+1 times, interpolation). */
pfmg_status pfmg_set_initial(pfmg_ctx *ctx, const double *u0, int32_t on_device);

/* One SDC sweep (eq. sdc-be / SDCcompactLIII) on slices [p_begin, p_end) of
 * level 0 (fine) or a coarser level 1 or 2 (right-hand side corrected by
 * that level's FAS term tau[m+1] - tau[m]; level 2 only in a three-level
 * context).  Slices are swept independently (their node-0 values are used
 * as they are).  Each node solve follows the solve policy.  PFMG_ERR_ARG
 * for a level the context does not have. */
pfmg_status pfmg_sdc_sweep(pfmg_ctx *ctx, int32_t level, int32_t p_begin, int32_t p_end);

/* Solve (I - alpha L_h) u = b on the fine grid with V-cycles (Sec. 4.1.1).
 * b, u: device pointers to n^dim float64; u is the initial guess and is
 * overwritten.  n_cycles > 0: that many cycles; 0: full solve (mg_tol,
 * mg_stall, mg_max_cycles).  *relres_out (may be NULL) receives
 * |b - H u|_inf / |b|_inf; *cycles_out (may be NULL) the cycles run.
 * Returns PFMG_STALLED / PFMG_NOT_CONVERGED for a full solve that stopped
 * early. */
pfmg_status pfmg_vcycle(pfmg_ctx *ctx, double alpha, const double *b, double *u,
                        int32_t n_cycles, double *relres_out, int32_t *cycles_out);

/* Static device scratch of pfmg_vcycle_noalloc, per GPU (64 MiB): enough
 * for a 3D FP64 solve up to n = 127 (the mixed form up to n = 63). */
#define PFMG_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * solve of pfmg_vcycle without a context or workspace.  It calls no
 * hipMalloc, hipFree, hipHostMalloc or other device-allocating routine;
 * its multigrid hierarchy and b / u staging live in a static device array
 * of PFMG_NOALLOC_SCRATCH_BYTES per GPU, held from the library's load until
 * the process ends.
 *   p: the grid and solve policy (dim, n, smoother, omega, nu_pre,
 *      nu_post, precision, stencil_order, mg_tol, mg_stall, mg_max_cycles;
 *      guess must be PFMG_GUESS_PREV; the time-stepping fields only need to
 *      pass pfmg_create's checks for a one-slice, one-level context).
 *   b, u: device pointers to n^dim float64 (C order, x fastest); u is the
 *      initial guess and is overwritten.  Borrowed for the call.
 *   n_cycles, relres_out, cycles_out: as pfmg_vcycle.
 *   hip_stream: the stream every launch goes to (NULL: the null stream).
 * With n_cycles > 0 and relres_out NULL the call only enqueues kernels on
 * the stream (stream-ordered, no synchronisation); otherwise it
 * synchronises the stream before returning.  PFMG_ERR_WORKSPACE (and
 * nothing launched) when the grid needs more scratch than the array holds;
 * PFMG_ERR_ARG for invalid parameters.  Every call on one GPU shares that
 * GPU's array and leaves its contents there: calls that overlap on one GPU
 * (other streams or threads) race and must be serialised by the caller. */
pfmg_status pfmg_vcycle_noalloc(const pfmg_params *p, double alpha, const double *b, double *u,
                                int32_t n_cycles, void *hip_stream, double *relres_out,
                                int32_t *cycles_out);

/* One IPFASST iteration (Sec. 2.4): new fine initial values from the
 * previous slices, fine sweeps on all slices, FAS restriction, coarse sweeps
 * in slice order, interpolation, collocation residual (three levels: with
 * middle-level sweeps after the restriction and after the coarse
 * correction).  *block_res_out (may be NULL) receives max over slices of
 * the residual (relative, or absolute with residual_abs). */
pfmg_status pfmg_pfasst_iter(pfmg_ctx *ctx, double *block_res_out);

/* Collocation residual (eq. resid) of every slice on level 0:
 * r[m] = U0_p - U[m] + dt sum_i Q[m][i] F[i] (m = 0..M), U0_p the previous
 * slice's end value (the block's initial value for p = 0);
 * per_slice_out[p] = max_m |r[m]|_inf / |U0_p|_inf (host array of P).
 * level must be 0.  PFMG_ERR_NAN if a value is NaN/Inf. */
pfmg_status pfmg_residual(pfmg_ctx *ctx, int32_t level, double *per_slice_out);

/* Run a whole block: set_initial (u0 as above), then iterations until the
 * block residual <= pfasst_tol or pfasst_max_iter.  Outputs (each may be
 * NULL): iterations run, final block residual.  PFMG_NOT_CONVERGED when
 * the cap was reached. */
pfmg_status pfmg_run_block(pfmg_ctx *ctx, const double *u0, int32_t on_device,
                           int32_t *iters_out, double *res_out);

/* Copy a field (PFMG_U_FINE .. PFMG_U_L2_OLD) of slice `slice`, node
 * `node` into / from a dense float64 array of its level's grid (n^dim on
 * the fine level, nc^dim on level 1, one more halving on level 2) on the
 * host (on_device == 0) or device. */
pfmg_status pfmg_get(pfmg_ctx *ctx, int32_t field, int32_t slice, int32_t node,
                     double *dst, int32_t on_device);
pfmg_status pfmg_set(pfmg_ctx *ctx, int32_t field, int32_t slice, int32_t node,
                     const double *src, int32_t on_device);

/* V-cycles run so far by node solves on level 0, 1 or 2 (counted per
 * slice; zero for a level the context does not have). */
pfmg_status pfmg_vcycle_count(pfmg_ctx *ctx, int32_t level, int64_t *count_out);

/* Kernel timing for measurement: while enabled, every launch of the named
 * kernel family ("<family>@<n>", e.g. "rbgs@127", "vcycle@127") is
 * bracketed by HIP events on the context's stream; the smoother's launches
 * carry events that the dispatch itself stamps (hipExtLaunchKernel), the
 * others events recorded around them.  Blocks run launch by launch (no
 * graph replay) while timing is on.  pfmg_timing_read returns the launches
 * recorded, their summed duration in milliseconds and the algorithmic bytes
 * they move (interior points times the per-point byte count of the kernel).
 * Enabling resets the counters; both calls synchronise the stream. */
pfmg_status pfmg_timing_enable(pfmg_ctx *ctx, const char *kernel, int32_t enable);
pfmg_status pfmg_timing_read(pfmg_ctx *ctx, int64_t *launches, double *ms_total,
                             double *bytes_total);

/* ------------------------------------------------------------------------
 * Batched form: many independent problems advanced together.
 *
 * The problems share every method parameter except n, nu and dt (the same
 * dim, slices, nodes, smoother, sweeps, omega, V-cycles per solve >= 1,
 * precision, pfasst_tol and pfasst_max_iter); each runs exactly the
 * algorithm of a single context.  Problems of one grid size form a group
 * and every kernel launch covers all groups (one launch per multigrid level
 * and leg for every (problem, slice) pair that has that level; the fused
 * red-black sweep's tile shape comes from the built-in autotuner).  After
 * the first call, block starts and iterations replay captured HIP graphs.
 * A problem whose block residual reaches pfasst_tol is frozen: later
 * iterations skip it, so its state stays the one at its own convergence.
 * At most 64 slices per problem.
 * ---------------------------------------------------------------------- */
typedef struct pfmg_batch pfmg_batch;

/* Device bytes for a batch of n_problems problems (per_problem[0..n-1]). */
pfmg_status pfmg_batch_workspace_bytes(const pfmg_params *per_problem, int32_t n_problems,
                                       size_t *bytes_out);
/* Create a batch; workspace and stream rules as for pfmg_create. */
pfmg_status pfmg_batch_create(const pfmg_params *per_problem, int32_t n_problems, void *workspace,
                              size_t bytes, void *hip_stream, pfmg_batch **out);
pfmg_status pfmg_batch_destroy(pfmg_batch *b);
/* Start a block for every problem: u0 holds the problems' dense initial
 * values one after the other in problem order (n_q^dim float64 each), on
 * the host or the device.  Runs each problem's predictor and makes every
 * problem active again. */
pfmg_status pfmg_batch_set_initial(pfmg_batch *b, const double *u0, int32_t on_device);
/* One IPFASST iteration of every active problem.  res_out (may be NULL,
 * else n_problems doubles) receives each problem's latest block residual
 * (frozen problems keep the value they converged with). */
pfmg_status pfmg_batch_pfasst_iter(pfmg_batch *b, double *res_out);
/* set_initial, then iterations until every problem is frozen or
 * pfasst_max_iter.  iters_out / res_out (may be NULL, else n_problems
 * entries): iterations each problem ran, its final block residual.
 * PFMG_NOT_CONVERGED if a problem did not reach pfasst_tol. */
pfmg_status pfmg_batch_run(pfmg_batch *b, const double *u0, int32_t on_device, int32_t *iters_out,
                           double *res_out);
/* As pfmg_get, for problem `problem`. */
pfmg_status pfmg_batch_get(pfmg_batch *b, int32_t problem, int32_t field, int32_t slice, int32_t node,
                           double *dst, int32_t on_device);
/* V-cycles run by node solves on level 0 / 1, summed over problems and
 * slices. */
pfmg_status pfmg_batch_vcycle_count(pfmg_batch *b, int32_t level, int64_t *count_out);
/* Launch timing as pfmg_timing_enable / pfmg_timing_read, for the batch's
 * one-pass red-black sweeps: family "rbgs@<n>", n the largest grid of a
 * multi-segment launch; the bytes count every segment's points. */
pfmg_status pfmg_batch_timing_enable(pfmg_batch *b, const char *kernel, int32_t enable);
pfmg_status pfmg_batch_timing_read(pfmg_batch *b, int64_t *launches, double *ms_total,
                                   double *bytes_total);

/* Streaming reference (measurement, not a step of the method): copy `bytes`
 * from src to dst, device pointers, with one 16-byte nontemporal load and
 * store per thread, the copy shape that streams fastest on gfx950.  The
 * benchmark times it next to the stencil kernels as the bandwidth HBM
 * delivers to a plain stream, and its hardware counters calibrate the
 * counter readings of the other kernels.  bytes and both pointers must be
 * multiples of 16 and the ranges must not overlap (PFMG_ERR_ARG).
 * Stream-ordered on hip_stream; does not synchronise. */
pfmg_status pfmg_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Red-black launch-shape autotuner: the number of configurations in the
 * process-wide table, and the entry for a key ("<arch>/rbgs/<f64|f32>/"
 * followed by n x fields per segment joined by '+'), written to buf as
 * "fused ty zchunk blocks" ("" if absent). */
pfmg_status pfmg_tune_count(int32_t *count_out);
pfmg_status pfmg_tune_lookup(const char *key, char *buf, size_t len);
/* Pins the table entry for a key of the form above, in place of timing:
 * every later red-black smoothing of that configuration in this process
 * takes it.  fused: 0 the two colour passes (ty, zchunk ignored); 1 the
 * one-pass kernel with 256-thread workgroups; 2 with 512; -1 drops the
 * entry, so that the next smoothing times the candidates.  ty: grid rows
 * per workgroup (1..n); zchunk: planes per z-chunk (>= 1).  PFMG_ERR_ARG for
 * a null or malformed key (n in 1..255 per segment) or a one-pass shape
 * without a compiled kernel: more than 6 rows per thread (ty + 2 rows over
 * threads / row lanes, row lanes = the widest n rounded up to 64), or more
 * than 3 with 512 threads.  The entry is not written to PFMG_TUNE_CACHE.
 * Thread-safe; a pin made while another thread smooths that configuration
 * takes effect from that thread's next smoothing. */
pfmg_status pfmg_tune_set(const char *key, int32_t fused, int32_t ty, int32_t zchunk);

/* ------------------------------------------------------------------------
 * Learned initial guess (a node solve's start from a small 3D network).
 *
 * A node solve (I - alpha L_h) u = b starts from the previous iterate U at
 * the node (Sec. 2.3.1).  The network maps r / |r|_inf, U / |U|_inf and
 * alpha (n+1)^2, with r = b - (I - alpha L_h) U, to y; its guess is
 * g = U + |r|_inf y.  The FP64 residual judges: a field takes g only if
 * |b - (I - alpha L_h) g|_inf < |r|_inf; the V-cycles of the full solve then
 * run from whichever start won.
 *
 * Network: a 3-level U-Net (widths 16/32/64) on the grids n, (n+1)/2 - 1,
 * ...: 3^3 convolutions with ReLU, stride-2 down and transposed up
 * convolutions (coarse point J on fine point 2J), skip concatenations and a
 * 1x1 output layer.  BF16 activations and weights on MFMA with FP32
 * accumulation; FP32 master weights and Adam for training.
 * Parameters (FP32, host): per layer in order W[cout][cin][3][3][3] (the
 * output layer W[1][16][1][1][1]) followed by b[cout].
 * ---------------------------------------------------------------------- */
typedef struct pfmg_nn pfmg_nn;

pfmg_status pfmg_nn_param_count(int64_t *count_out);
/* Device bytes of a network for grid n (odd with odd coarse grids down to
 * >= 3 points on the third level) and up to `batch` samples per call;
 * training adds gradients, Adam moments and gradient tensors. */
pfmg_status pfmg_nn_workspace_bytes(int32_t n, int32_t batch, int32_t training, size_t *bytes_out);
pfmg_status pfmg_nn_create(int32_t n, int32_t batch, int32_t training, void *workspace, size_t bytes,
                           void *hip_stream, pfmg_nn **out);
pfmg_status pfmg_nn_destroy(pfmg_nn *nn);
/* Set / read the parameters (host arrays of pfmg_nn_param_count floats);
 * loading resets the Adam state. */
pfmg_status pfmg_nn_load(pfmg_nn *nn, const float *params, int64_t count);
pfmg_status pfmg_nn_save(pfmg_nn *nn, float *params, int64_t count);
/* He-normal weights (std sqrt(2 / fan_in); the output layer 0.1 of that),
 * zero biases, from a counter-based generator seeded by `seed`. */
pfmg_status pfmg_nn_init(pfmg_nn *nn, uint64_t seed);
/* Forward pass on dense inputs x [batch][3][n^3] (device FP32): y
 * [batch][n^3] (device FP32). */
pfmg_status pfmg_nn_forward(pfmg_nn *nn, const float *x, int32_t batch, float *y);
/* Mean squared error against target [batch][n^3] (device) and its
 * gradient with respect to every parameter (host, parameter layout). */
pfmg_status pfmg_nn_gradients(pfmg_nn *nn, const float *x, const float *target, int32_t batch,
                              double *loss_out, float *grads_out);
/* One Adam step (lr; betas 0.9, 0.999; eps 1e-8) on the recorded pairs
 * idx[0..batch-1] (host indices, each in 0..n_pairs-1) of a pair store of
 * n_pairs pairs (see pfmg_record).  *loss_out: the batch's mean squared
 * error before the step. */
pfmg_status pfmg_nn_train_step(pfmg_nn *nn, const void *pairs, const float *ah2, int32_t n_pairs,
                               const int32_t *idx, int32_t batch, float lr, double *loss_out);
/* Copy of a layer's tensor from the last forward / backward pass to dense
 * device FP32 [batch][channels][n_l^3]: which = 0 input, 1 output, 2
 * gradient of the pre-activation (after the ReLU mask), 3 gradient of the
 * input.  Layers 0..12 (the 3^3 convolutions). */
pfmg_status pfmg_nn_tensor(pfmg_nn *nn, int32_t layer, int32_t which, int32_t batch, float *dst);
/* Use `nn` (or none: NULL) for the fine-level node solves of a context
 * created with guess = PFMG_GUESS_LEARNED (3D, full solves).  The network's
 * grid must be the context's fine grid and its batch >= n_slices; it runs
 * on the context's stream. */
pfmg_status pfmg_attach_nn(pfmg_ctx *ctx, pfmg_nn *nn);
/* Fields offered the learned guess and fields that took it. */
pfmg_status pfmg_guess_stats(pfmg_ctx *ctx, int64_t *tried, int64_t *taken);
/* Record training pairs from the fine-level full node solves of a 3D
 * context (vcycles_per_solve = 0): pair k gets BF16 dense [3][n^3] at
 * pairs + 3 k n^3 (r / |r|, U / |U| before the solve, (u - U) / |r| after
 * it) and FP32 alpha (n+1)^2 at ah2[k].  scratch: device FP64
 * [n_slices][n^3].  Recording stops when `capacity` pairs are full; NULL
 * pairs turns it off.  Device pointers stay owned by the caller. */
pfmg_status pfmg_record(pfmg_ctx *ctx, void *pairs, float *ah2, double *scratch, int32_t capacity);
pfmg_status pfmg_record_count(pfmg_ctx *ctx, int32_t *count_out);

#ifdef __cplusplus
}
#endif
#endif
