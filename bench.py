"""Benchmark: seconds to a 1e-10 relative residual per PFASST block.

Workload (one step = one whole block): 3D heat equation u_t = Laplace(u) on
the unit cube, Dirichlet 0, 127^3 interior points, initial data a product of
sines plus 32 seeded random sine modes (seed 1407); IPFASST with 16 time
slices of dt = 1e-3, 5 / 3 Gauss-Lobatto nodes, coarse grid 63^3,
red-black Gauss-Seidel V(2,2) node solves with one V-cycle per solve, FP64;
predictor, then iterations until the block residual is <= 1e-10.

The initial data sits in HBM before the timed region, which runs whole
blocks as the library does (captured graphs replayed per iteration).
Printed: one JSON line with the block time, V-cycle GDOF/s, the roofline of
the dominant kernel (the one-pass red-black sweep on the fine grid, its
launches stamping HIP events on the stream they run on during one more
block of the same workload in a context whose coarse chain shares the main
stream, and again beside the chain in the benchmark's own context; HBM
traffic from the committed counter summary while the kernel source and
launch shape are unchanged) and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense


def stamped_roofline(ctx, u0, family, n):
    """One more block with the launches of kernel family `family` at grid n
    bracketed by dispatch-stamped events: algorithmic bytes per launch over
    the average launch duration."""
    ctx.timing_enable(f"{family}@{n}", True)
    ctx.run_block(u0)
    launches, ms, nbytes = ctx.timing_read()
    ctx.timing_enable(None, False)
    if launches == 0 or ms <= 0:
        return None
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": f"{family}@{n}",
            "launches": launches, "avg_launch_us": round(ms * 1e3 / launches, 2), "bytes_per_launch": nbytes / launches}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=127)
    ap.add_argument("--slices", type=int, default=16)
    ap.add_argument("--vcycles", type=int, default=1, help="V-cycles per solve (0 = full solve)")
    ap.add_argument("--smoother", choices=["rbgs", "jacobi"], default="rbgs")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2, help="oracle iterations in the CPU sample")
    ap.add_argument("--max-iter", type=int, default=400,
                    help="iteration cap per block (profiling runs cap it to keep traces small)")
    ap.add_argument("--form", choices=["mixed", "batched", "learned", "nn-forward", "solve-policies", "heat1d", "table1",
                                       "weak3"],
                    default=None,
                    help="instead: one of the method's forms against the plain FP64 path (mixed, batched, learned), "
                         "the network's forward pass alone (nn-forward), "
                         "the node-solve policies at 127^3 x 16 (solve-policies), the 1D latency and error report "
                         "(heat1d) or the paper's 3D strong-scaling problem with its uniform nodes, ISDC / IMLSDC / "
                         "IPFASST (table1)")
    ap.add_argument("--table1-config", choices=["2nd/2nd", "2nd/4th", "4th/4th"], default=None,
                    help="with --form table1: only this temporal-order configuration")
    ap.add_argument("--table1-f", choices=["solve-interp", "plain"], default="solve-interp",
                    help="with --form table1: F from the node solves and interpolated coarse F changes "
                         "(f_solve = f_interp = 1), or F = nu L U throughout")
    ap.add_argument("--table1-tol", choices=["absolute", "relative"], default="absolute",
                    help="with --form table1: the 1e-9 residual bound on the max-norm residual, or relative to "
                         "the slice's initial value")
    ap.add_argument("--cpu-full-block", action="store_true",
                    help="instead: run the oracle's whole block to 1e-10 on the host (minutes) and print its time")
    ap.add_argument("--families", action="store_true",
                    help="also report every kernel family's launches, event-stamped time and algorithmic bytes "
                         "per launch on the fine (127) and coarse (63) grid, one more block per family")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run the library's streaming copy of 1 GiB three times (reference for the HBM "
                         "counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rbgs_fused_127x16_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1407_6486_amd", "csrc", "rbgs_fused.hip")


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or the kernel source changed since."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            lines = [ln for ln in f if ln.startswith("bench-traffic: ")]
        rec = json.loads(lines[-1][len("bench-traffic: "):])
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != sha:
        return None
    return rec


CALIB_BYTES = 1 << 30


def copy_calibration(pfmg):
    """A plain copy of known size for the HBM counters: the library's
    streaming copy of 1 GiB, three times (per dispatch 1 GiB read, 1 GiB
    written)."""
    import torch

    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        pfmg.pfmg_stream_copy(b.data_ptr(), a.data_ptr(), CALIB_BYTES, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def host_info():
    """The host the oracle runs on: CPU model, sockets x cores per socket
    (physical cores) and logical CPUs from lscpu."""
    import subprocess

    info = {"model": None, "physical_cores": None, "logical_cpus": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {ln.split(":", 1)[0].strip(): ln.split(":", 1)[1].strip() for ln in out.splitlines() if ":" in ln}
        info["model"] = kv.get("Model name")
        if kv.get("Socket(s)", "").isdigit() and kv.get("Core(s) per socket", "").isdigit():
            info["physical_cores"] = int(kv["Socket(s)"]) * int(kv["Core(s) per socket"])
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def host_triad_gbs(threads, nbytes=1 << 29, reps=5):
    """STREAM-triad bandwidth of the host (a = b + s c over three arrays of
    nbytes, one fused pass on `threads` threads; 3 nbytes moved per pass)."""
    import torch

    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    b = torch.ones(nbytes // 8, dtype=torch.float64)
    c = torch.ones_like(b)
    a = torch.empty_like(b)
    torch.add(b, c, alpha=3.0, out=a)
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.add(b, c, alpha=3.0, out=a)
    dt = (time.perf_counter() - t0) / reps
    torch.set_num_threads(prev)
    return 3 * nbytes / dt / 1e9


def _omp_threads(k):
    """Set the OpenMP thread count of the oracle's runtime (libgomp)."""
    import ctypes

    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))


def cpu_baseline(n, P, iters_gpu, cpu_iters, u0):
    """The oracle as it stands (gcc -O3, no fast-math, no contraction), on
    the host: predictor + cpu_iters iterations on the threads of the
    process's CPU share (OMP_NUM_THREADS), extrapolated to the iteration count of the
    block; then the same on one thread (predictor + one iteration); the
    host's CPU model, physical cores and STREAM-triad bandwidth."""
    import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def sample(k, iters):
        _omp_threads(k)
        t0 = time.perf_counter()
        orc = O.Pfasst(3, n, 1.0, 1e-3, P, 5, 3, O.policy(cycles=1))
        orc.set_initial(u0)
        t1 = time.perf_counter()
        for _ in range(iters):
            orc.iterate()
        t2 = time.perf_counter()
        return t1 - t0, (t2 - t1) / iters

    pred, per_iter = sample(threads, cpu_iters)
    pred1, per_iter1 = sample(1, 1)
    _omp_threads(threads)
    est = pred + per_iter * iters_gpu
    est1 = pred1 + per_iter1 * iters_gpu
    host = host_info()
    host["threads_used"] = threads
    host["triad_gbs"] = round(host_triad_gbs(threads), 1)
    host["triad_gbs_one_thread"] = round(host_triad_gbs(1), 1)
    return {"value": round(est, 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"predictor ({pred:.2f} s) + {cpu_iters} iterations ({per_iter:.2f} s each) of the "
                      f"same block on {threads} threads, extrapolated to the {iters_gpu} iterations the block needs",
            "one_thread": {"value": round(est1, 3), "sample": f"predictor ({pred1:.2f} s) + 1 iteration "
                                                               f"({per_iter1:.2f} s) on 1 thread, extrapolated"},
            "host": host}


def cpu_full_block(n, P, u0, tol=1e-10, max_iter=400):
    """The oracle's whole block to the residual bound (validates the
    extrapolation of cpu_baseline); prints a progress line every 10
    iterations."""
    import oracle as O

    t0 = time.perf_counter()
    orc = O.Pfasst(3, n, 1.0, 1e-3, P, 5, 3, O.policy(cycles=1))
    orc.set_initial(u0)
    it, res = 0, float("inf")
    while it < max_iter and res > tol:
        res = orc.iterate()
        it += 1
        if it % 10 == 0:
            print(f"oracle block: iteration {it} residual {res:.3e} at {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    return {"value": round(time.perf_counter() - t0, 3), "unit": "s", "iterations": it, "final_residual": res,
            "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}


def copy_bandwidth_gbs(pfmg, nbytes=1 << 30, reps=10):
    """Read + write bytes per second of the library's streaming copy of
    nbytes (one 16-byte nontemporal load and store per thread), timed with
    HIP events on the stream it runs on: the bandwidth a plain stream gets
    from HBM on this GPU, next to the 8 TB/s spec peak."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(3):
        pfmg.pfmg_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, st.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        pfmg.pfmg_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, st.cuda_stream)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _time_blocks(run, steps):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [run() for _ in range(steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def form_mixed(pfmg, a):
    """255^3, 16 slices (seed 1408): FP32 multigrid inside FP64 refinement
    against the FP64 path, both to a block residual of 1e-10."""
    import torch

    import inputs

    n, P = 255, 16
    u0 = torch.from_numpy(inputs.random_fourier(n, 1408)[0]).to("cuda")
    res = {}
    for prec in ("fp64", "mixed"):
        c = pfmg.Context(pfmg.pfmg_default_params(n=n, n_slices=P, pfasst_tol=1e-10, pfasst_max_iter=a.max_iter,
                                                   precision=pfmg.MIXED if prec == "mixed" else pfmg.FP64))
        for _ in range(a.warmup):
            c.run_block(u0)
        t, outs = _time_blocks(lambda: c.run_block(u0), a.steps)
        res[prec] = (t, outs[-1][1], outs[-1][2], stamped_roofline(c, u0, "rbgs", n))
        c.close()
        del c
        torch.cuda.empty_cache()
    return {"metric": "s to 1e-10 residual per PFASST block", "value": round(res["mixed"][0], 4), "unit": "s",
            "form": "mixed precision (FP32 multigrid in FP64 refinement)", "plain_value": round(res["fp64"][0], 4),
            "speedup_vs_plain": round(res["fp64"][0] / res["mixed"][0], 3),
            "iterations": {"mixed": res["mixed"][1], "fp64": res["fp64"][1]},
            "final_residual": {"mixed": res["mixed"][2], "fp64": res["fp64"][2]},
            "roofline": res["mixed"][3], "roofline_fp64_path": res["fp64"][3],
            "higher_is_better": False, "dtype": "f64+f32", "data": "synthetic", "n_gpus": 1, "steps": a.steps,
            "config": {"workload": "3D heat, 255^3, 16 slices, dt=1e-3, Lobatto 5/3, rbgs V(2,2), 1 V-cycle/solve, "
                                   "seed 1408"}}


def form_batched(pfmg, a):
    """64 uneven problems (n in {31, 63, 95, 127}, nu and dt log-uniform,
    P = 4): one batch against a loop over 64 single contexts."""
    import torch

    import inputs

    probs = [inputs.batch_problem(q) for q in range(64)]
    ps = [pfmg.pfmg_default_params(n=bp.n, nu=bp.nu, dt=bp.dt, n_slices=4, pfasst_tol=1e-10, pfasst_max_iter=1000)
          for bp in probs]
    u0s = [torch.from_numpy(bp.u0).to("cuda") for bp in probs]
    b = pfmg.Batch(ps)
    for _ in range(a.warmup):
        b.run(u0s)
    tb, outs = _time_blocks(lambda: b.run(u0s), a.steps)
    its = outs[-1][1]
    b.close()
    del b
    torch.cuda.empty_cache()
    # the batch's dominant sweeps (launches whose largest grid is 127^3),
    # timed on a block of 6 iterations in which no problem stops early, so
    # that every launch covers all fields (the byte count assumes it)
    pr = [pfmg.pfmg_default_params(n=bp.n, nu=bp.nu, dt=bp.dt, n_slices=4, pfasst_tol=0.0, pfasst_max_iter=6)
          for bp in probs]
    b = pfmg.Batch(pr)
    b.run(u0s)
    b.timing_enable("rbgs@127", True)
    b.run(u0s)
    nl, ms, nbytes = b.timing_read()
    b.timing_enable(None, False)
    roof = None
    if nl and ms > 0:
        ach = nbytes / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "rbgs@127 (multi-segment one-pass sweeps led by the 127^3 problems; 6-iteration block, "
                          "no problem frozen)", "launches": nl,
                "avg_launch_us": round(ms * 1e3 / nl, 2), "bytes_per_launch": nbytes / nl}
    b.close()
    del b
    torch.cuda.empty_cache()
    ctxs = [pfmg.Context(p) for p in ps]
    for c, u in zip(ctxs, u0s):
        c.run_block(u)
    tl, _ = _time_blocks(lambda: [c.run_block(u) for c, u in zip(ctxs, u0s)], 1)
    for c in ctxs:
        c.close()
    dof = sum(bp.n ** 3 for bp in probs)
    return {"metric": "s to 1e-10 residual per PFASST block", "value": round(tb, 4), "unit": "s",
            "form": "batched (64 uneven problems, shared multi-segment launches, graphs)",
            "plain_value": round(tl, 4), "plain": "loop over 64 single contexts",
            "speedup_vs_plain": round(tl / tb, 3), "iterations_min_max": [int(its.min()), int(its.max())],
            "roofline": roof,
            "higher_is_better": False, "dtype": "f64", "data": "synthetic", "n_gpus": 1, "steps": a.steps,
            "config": {"workload": f"64 problems, n in {{31,63,95,127}}, {dof / 1e6:.1f} M DOF per slice, P=4, "
                                   "nu 10^U(-1,1), dt 10^U(-4,-2), seeds [6486, q]"}}


def form_learned(pfmg, a):
    """Learned initial guess: record 20k pairs at 63^3, train, evaluate at
    127^3 with 16 slices and full node solves against the plain guess."""
    import numpy as np

    from paper_1407_6486_amd import learned as L

    # progress on stderr (the stdout line stays the JSON result)
    quiet = lambda m: print(m, file=sys.stderr, flush=True)
    store, count = L.record(pfmg, 63, 20000, log=quiet)
    net, losses, t_train = L.train(pfmg, store, count, 2000, 8, 2e-3, log=quiet)
    params = net.save()
    net.close()
    del store
    t_inf = L.inference_time(pfmg, params, 127, 16)
    ev = L.evaluate(pfmg, params, 127, 16, (0.0, 1e-4), log=quiet)
    # the other plain path: the benchmark's one V-cycle per node solve
    import inputs
    import torch
    c1 = pfmg.Context(pfmg.pfmg_default_params(n=127, n_slices=16, pfasst_tol=1e-10, pfasst_max_iter=400))
    u0 = torch.from_numpy(inputs.random_fourier(127, 1407)[0]).to("cuda")
    c1.run_block(u0)
    v0 = c1.vcycle_count(0)
    s_one, out_one = _time_blocks(lambda: c1.run_block(u0), 2)
    one_v = {"s_per_block": round(s_one, 4), "iterations": out_one[-1][1], "residual": out_one[-1][2],
             "fine_vcycles": (c1.vcycle_count(0) - v0) // 2}
    c1.close()
    best = min((k for k in ev if k != "plain"), key=lambda k: ev[k]["s_per_block"])
    return {"metric": "s to 1e-10 residual per PFASST block", "value": round(ev[best]["s_per_block"], 4),
            "unit": "s", "form": f"learned initial guess ({best})", "plain_value": round(ev["plain"]["s_per_block"], 4),
            "speedup_vs_plain": round(ev["plain"]["s_per_block"] / ev[best]["s_per_block"], 3),
            "plain_one_vcycle": one_v,
            "speedup_vs_plain_one_vcycle": round(one_v["s_per_block"] / ev[best]["s_per_block"], 3),
            "eval": ev, "train_pairs": count, "train_steps": 2000, "train_s": round(t_train, 1),
            "loss_first_last": [float(np.mean(losses[:50])), float(np.mean(losses[-50:]))],
            "inference_ms_16x127": round(t_inf * 1e3, 2),
            "inference_tflops": round(L.flops_per_voxel() * 127 ** 3 * 16 / t_inf / 1e12, 1),
            "roofline": {"bound": "mfma", "kernel": "network forward, 16 x 127^3 (BF16 MFMA, FP32 accumulate)",
                         "achieved": round(L.flops_per_voxel() * 127 ** 3 * 16 / t_inf / 1e12, 1),
                         "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(L.flops_per_voxel() * 127 ** 3 * 16 / t_inf / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4),
                         "traffic": None},
            "higher_is_better": False, "dtype": "f64 solver, bf16 network", "data": "synthetic", "n_gpus": 1,
            "config": {"workload": "train 63^3 (seeds [20000, r], dt 10^U(-3,-2), P=4); evaluate 127^3, 16 slices, "
                                   "dt=1e-3, seed 1407, full solves to 1e-12"}}


def form_nn_forward(pfmg, a):
    """The learned guess's network alone: forward passes of 16 x 127^3 with
    randomly initialised weights on a seeded random input (the timing does
    not depend on the values)."""
    import torch

    from paper_1407_6486_amd import learned as L

    if a.calibrate_copy:
        copy_calibration(pfmg)
    n, batch = 127, 16
    net = pfmg.Net(n, batch, training=False)
    net.init(1407)
    g = torch.Generator(device="cuda").manual_seed(1407)
    x = torch.randn((batch, 3, n ** 3), dtype=torch.float32, device="cuda", generator=g)
    y = torch.empty((batch, n ** 3), dtype=torch.float32, device="cuda")
    for _ in range(max(a.warmup, 1)):
        pfmg.pfmg_nn_forward(net.h, x.data_ptr(), batch, y.data_ptr())
    torch.cuda.synchronize()
    reps = max(a.steps, 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        pfmg.pfmg_nn_forward(net.h, x.data_ptr(), batch, y.data_ptr())
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    net.close()
    tf = L.flops_per_voxel() * n ** 3 * batch / t / 1e12
    return {"metric": "ms per network forward pass", "value": round(t * 1e3, 3), "unit": "ms",
            "form": "learned guess network forward", "steps": reps, "warmup": max(a.warmup, 1),
            "roofline": {"bound": "mfma", "kernel": "network forward, 16 x 127^3 (BF16 MFMA, FP32 accumulate)",
                         "achieved": round(tf, 1), "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / BF16_MFMA_PEAK_TFLOPS, 4), "traffic": None},
            "higher_is_better": False, "dtype": "bf16", "data": "synthetic", "n_gpus": 1,
            "config": {"workload": "U-Net 16/32/64, 16 x 127^3, random weights (seed 1407), random input"}}


def form_solve_policies(pfmg, a):
    """The 127^3 x 16 block (seed 1407) with the node-solve policies the
    paper weighs against each other: one and two V-cycles per solve and
    full solves (1e-12, stall 0.75), red-black Gauss-Seidel; one V-cycle
    with omega-Jacobi (2/3).  Each to a block residual of 1e-10."""
    import torch

    import inputs

    n, P = 127, 16
    u0 = torch.from_numpy(inputs.random_fourier(n, 1407)[0]).to("cuda")
    rows = []
    for sm, cyc in (("rbgs", 1), ("rbgs", 2), ("rbgs", 0), ("jacobi", 1)):
        c = pfmg.Context(pfmg.pfmg_default_params(
            dim=3, n=n, n_slices=P, nu=1.0, dt=1e-3, vcycles_per_solve=cyc, mg_tol=1e-12, mg_stall=0.75,
            mg_max_cycles=50, smoother=pfmg.SMOOTH_RBGS if sm == "rbgs" else pfmg.SMOOTH_JACOBI,
            omega=1.0 if sm == "rbgs" else 2.0 / 3.0, pfasst_tol=1e-10, pfasst_max_iter=a.max_iter))
        for _ in range(max(1, a.warmup)):
            c.run_block(u0)
        v0 = c.vcycle_count(0)
        t, outs = _time_blocks(lambda: c.run_block(u0), a.steps)
        fine = (c.vcycle_count(0) - v0) / a.steps
        c.timing_enable(f"vcycle@{n}", True)
        c.run_block(u0)
        _, vms, vdof = c.timing_read()
        c.timing_enable(None, False)
        rows.append({"smoother": sm, "vcycles_per_solve": cyc if cyc else "to 1e-12", "s_per_block": round(t, 4),
                     "iterations": outs[-1][1], "final_residual": outs[-1][2], "fine_vcycles_per_block": fine,
                     "vcycle_gdofs": round(vdof / (vms * 1e-3) / 1e9, 2) if vms > 0 else None})
        c.close()
        del c
        torch.cuda.empty_cache()
    return {"metric": "s to 1e-10 residual per PFASST block", "unit": "s", "form": "node-solve policies",
            "rows": rows, "higher_is_better": False, "dtype": "f64", "data": "synthetic", "n_gpus": 1,
            "steps": a.steps, "config": {"workload": "3D heat, 127^3, 16 slices, dt=1e-3, Lobatto 5/3, V(2,2), "
                                                     "seed 1407"}}


def form_heat1d(pfmg, a):
    """1D heat (n = 127, sin(pi x) + 0.1 sin(8 pi x), nu = 1), 4 slices of
    dt = 0.01, omega-Jacobi V(2,2), one V-cycle per solve: predictor and 5
    iterations.  Per iteration the block residual and, over the slice ends,
    the error against the semi-discrete (ODE) solution, whose sine modes
    decay as exp(mu_k t), mu_k = -4 sin^2(k pi h / 2) / h^2, and against the
    PDE solution (exp(-k^2 pi^2 t)).  A latency test: s per block."""
    import numpy as np

    n, P, dt = 127, 4, 0.01
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u0 = np.sin(np.pi * x) + 0.1 * np.sin(8 * np.pi * x)
    mu = lambda k: -4.0 * np.sin(k * np.pi * h / 2) ** 2 / h ** 2
    ode = lambda t: np.exp(mu(1) * t) * np.sin(np.pi * x) + 0.1 * np.exp(mu(8) * t) * np.sin(8 * np.pi * x)
    pde = lambda t: (np.exp(-np.pi ** 2 * t) * np.sin(np.pi * x)
                     + 0.1 * np.exp(-64 * np.pi ** 2 * t) * np.sin(8 * np.pi * x))
    kw = dict(dim=1, n=n, n_slices=P, nu=1.0, dt=dt, smoother=pfmg.SMOOTH_JACOBI, omega=2.0 / 3.0,
              vcycles_per_solve=1, pfasst_tol=0.0, pfasst_max_iter=5)
    c = pfmg.Context(pfmg.pfmg_default_params(**kw))
    c.set_initial(u0)

    def errors():
        ends = [c.get(pfmg.U_FINE, p, 4) for p in range(P)]
        e_ode = max(float(np.max(np.abs(u - ode((p + 1) * dt)))) for p, u in enumerate(ends))
        e_pde = max(float(np.max(np.abs(u - pde((p + 1) * dt)))) for p, u in enumerate(ends))
        return e_ode, e_pde

    per_iter = [{"iteration": 0, "residual": float(np.max(c.residual())), **dict(zip(("ode_error", "pde_error"),
                                                                                   errors()))}]
    for k in range(1, 6):
        r = c.pfasst_iter()
        per_iter.append({"iteration": k, "residual": r, **dict(zip(("ode_error", "pde_error"), errors()))})
    c.close()
    c = pfmg.Context(pfmg.pfmg_default_params(**kw))
    for _ in range(max(1, a.warmup)):
        c.run_block(u0)
    t, _ = _time_blocks(lambda: c.run_block(u0), max(a.steps, 10))
    c.close()
    return {"metric": "s per PFASST block (predictor + 5 iterations)", "value": round(t, 6), "unit": "s",
            "form": "1D heat, latency and errors", "per_iteration": per_iter, "higher_is_better": False, "dtype": "f64",
            "data": "synthetic", "n_gpus": 1,
            "config": {"workload": "1D heat, n=127, 4 slices, dt=0.01, Lobatto 5/3, jacobi V(2,2), 1 V-cycle/solve"}}


# Table 1 of Sec. 4.3 (speedup of IPFASST over ISDC with the same spatial
# resources; N_p = 1 is IMLSDC), for context next to the single-GPU figures.
PAPER_TABLE1 = {
    "2nd/2nd": {1: 0.8, 2: 1.2, 4: 2.1, 8: 3.5, 16: 5.6, 32: 8.6},
    "2nd/4th": {1: 0.9, 2: 1.4, 4: 2.6, 8: 4.6, 12: 5.9, 24: 7.2},
    "4th/4th": {1: 0.7, 2: 1.0, 4: 1.9, 8: 3.2, 12: 4.6, 24: 6.6},
}


def form_weak3(pfmg, a):
    """Sec. 4.2's weak-scaling runs: 1D heat, nu = L = T = 1, u0 = sin(pi x),
    N_x = N_t = 32, 64, 128 (n = N - 1 interior points, N slices of one
    block), three levels coarsened by two in space, uniform nodes (3 on the
    fine and middle levels, backward Euler on the coarsest), two red-black
    V(2,2) cycles per solve, both F options and cubic interpolation; the
    two-level hierarchy beside it.  Per iteration: the last slice's error
    against exp(-pi^2) sin(pi x) (PDE) and against the semi-discrete
    solution (ODE), and the block residual; the wall time of the iterations
    to the error level (the first iteration within 10 % of the converged
    error, which 30 iterations give)."""
    import numpy as np

    out = {}
    for N in (32, 64, 128):
        n = N - 1
        h = 1.0 / N
        x = np.arange(1, n + 1) * h
        u0 = np.sin(np.pi * x)
        pde = np.exp(-np.pi ** 2) * u0
        ode = np.exp(-4.0 * np.sin(np.pi * h / 2) ** 2 / h ** 2) * u0
        for levels in (3, 2):
            c = pfmg.Context(pfmg.pfmg_default_params(
                dim=1, n=n, nu=1.0, dt=1.0 / N, n_slices=N, nodes_fine=3, nodes_coarse=2,
                nodes_middle=3 if levels == 3 else 0, node_family=pfmg.NODES_UNIFORM, smoother=pfmg.SMOOTH_RBGS,
                omega=1.0, vcycles_per_solve=2, interp_order=4, f_solve=1, f_interp=1))
            c.set_initial(u0)
            rows = []
            for k in range(30):
                r = c.pfasst_iter()
                ue = c.get(pfmg.U_FINE, N - 1, 2)
                rows.append((float(np.max(np.abs(ue - pde))), float(np.max(np.abs(ue - ode))), r))
            level = rows[-1][0]
            reach = next(k + 1 for k, (e, _, _) in enumerate(rows) if abs(e - level) <= 0.1 * level)
            c.set_initial(u0)
            import torch
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reach):
                c.pfasst_iter()
            torch.cuda.synchronize()
            out[f"N={N}, {levels} levels"] = {
                "iteration_reaching_error_level": reach, "s_to_level": round(time.perf_counter() - t0, 5),
                "pde_error": [float(f"{e:.3e}") for e, _, _ in rows[:8]],
                "ode_error": [float(f"{o:.3e}") for _, o, _ in rows[:8]],
                "residual": [float(f"{q:.3e}") for _, _, q in rows[:8]], "converged_pde_error": float(f"{level:.4e}")}
            c.close()
    return {"metric": "iterations to the error level (Sec. 4.2 weak scaling, N=128, three levels)",
            "value": out["N=128, 3 levels"]["iteration_reaching_error_level"], "unit": "iterations",
            "form": "three-level IPFASST, N_x = N_t", "runs": out, "paper": "error level at iteration 5 (N=32), 3 (N=64, 128)",
            "higher_is_better": False, "dtype": "f64", "data": "synthetic", "n_gpus": 1,
            "config": {"workload": "1D heat, nu=1, T=1, sin(pi x), N_x=N_t=32/64/128 (N slices), uniform nodes 3/3/2, "
                                   "rbgs V(2,2), 2 V-cycles/solve, cubic interpolation, F options"}}


def form_table1(pfmg, a):
    """The 3D strong-scaling problem of Sec. 4.3 (nu = 1/3, T = 1,
    u0 = sin(pi x) sin(pi y) sin(pi z), zero Dirichlet data), with the
    paper's uniform nodes whose quadrature leaves out the left end point:
    second order in space and time (127^3, 3 fine nodes over backward
    Euler, 128 steps), second order in space and fourth in time (127^3, 5
    fine nodes over 3, 24 steps), fourth order in both (31^3 with the
    fourth-order fine stencil over a second-order 15^3 coarse level, 24
    steps).  The two-level methods interpolate in space with cubics, as the
    paper's runs do.  Each solve is two V(2,2) red-black cycles; F at a
    node comes from its solve and the fine F values take the interpolated
    coarse F change (f_solve, f_interp; --table1-f plain re-evaluates F =
    nu L U instead).  Each step or block iterates until every slice's
    residual is at most 1e-9 in the max-norm (residual_abs;
    --table1-tol relative: relative to the slice's initial value), at most
    50 iterations.  On one GPU the paper's time
    ranks become slices of one block, advanced together: serial ISDC (one
    level, one slice a block), serial IMLSDC (two levels, one slice) and
    IPFASST with N_p slices a block are timed over the whole interval, and
    the speedup over ISDC is reported next to the paper's Table 1.  Errors
    are the max-norm distance of the final state to the PDE solution
    exp(-pi^2 T) sin sin sin and to the semi-discrete one."""
    import numpy as np
    import torch

    import inputs

    nu, T = 1.0 / 3.0, 1.0
    configs = {"2nd/2nd": dict(n=127, so=2, nf=3, nc=2, steps=128, nps=(2, 4, 8, 16, 32)),
               "2nd/4th": dict(n=127, so=2, nf=5, nc=3, steps=24, nps=(2, 4, 8, 12, 24)),
               "4th/4th": dict(n=31, so=4, nf=5, nc=3, steps=24, nps=(2, 4, 8, 12, 24))}
    if a.table1_config:
        configs = {k: v for k, v in configs.items() if k == a.table1_config}
    out = {}
    for name, cf in configs.items():
        n = cf["n"]
        h = 1.0 / (n + 1)
        u0 = torch.from_numpy(inputs.sine_mode(n, (1, 1, 1), 3)).to("cuda")
        shape0 = inputs.sine_mode(n, (1, 1, 1), 3)
        pde = np.exp(-np.pi ** 2 * T) * shape0
        # the semi-discrete solution: the sine mode decays with the stencil's eigenvalue
        if cf["so"] == 4:
            mu = 3 * (-2 * np.cos(2 * np.pi * h) + 32 * np.cos(np.pi * h) - 30) / (12 * h * h)
        else:
            mu = 3 * (-4.0 * np.sin(np.pi * h / 2) ** 2 / h ** 2)
        ode = np.exp(nu * mu * T) * shape0
        dt = T / cf["steps"]
        rows = []
        runs = [("ISDC", 1, 0)] + [("IMLSDC", 1, cf["nc"])] + [("IPFASST", npr, cf["nc"]) for npr in cf["nps"]]
        fopt = 1 if a.table1_f == "solve-interp" else 0
        for kind, P, nc in runs:
            c = pfmg.Context(pfmg.pfmg_default_params(
                dim=3, n=n, nu=nu, dt=dt, n_slices=P, nodes_fine=cf["nf"], nodes_coarse=nc,
                node_family=pfmg.NODES_UNIFORM, smoother=pfmg.SMOOTH_RBGS, omega=1.0, vcycles_per_solve=2,
                pfasst_tol=1e-9, pfasst_max_iter=50, stencil_order=cf["so"], interp_order=4 if nc else 2,
                f_solve=fopt, f_interp=fopt if nc else 0, residual_abs=int(a.table1_tol == "absolute")))
            nblocks = cf["steps"] // P

            def interval():
                u, its, ok = u0, [], True
                for _ in range(nblocks):
                    st, it, _ = c.run_block(u)
                    its.append(it)
                    ok = ok and st == pfmg.OK
                    u = c.get(pfmg.U_FINE, P - 1, cf["nf"] - 1, host=False)
                return u, its, ok

            for _ in range(max(1, a.warmup)):
                interval()
            t, outs = _time_blocks(interval, max(1, a.steps))
            u_end, its, ok = outs[-1]
            ue = u_end.cpu().numpy()
            rows.append({"method": kind, "n_p": P, "blocks": nblocks, "s": round(t, 4), "converged": ok,
                         "iterations_per_block": round(float(np.mean(its)), 2), "iterations_max": int(max(its)),
                         "pde_error": float(np.max(np.abs(ue - pde))), "ode_error": float(np.max(np.abs(ue - ode)))})
            c.close()
            del c
            torch.cuda.empty_cache()
        t_isdc = rows[0]["s"]
        for r in rows:
            r["speedup_vs_isdc"] = round(t_isdc / r["s"], 3)
            r["paper_speedup"] = PAPER_TABLE1[name].get(r["n_p"]) if r["method"] != "ISDC" else None
        out[name] = rows
    conv = [(r["s"], name, r["method"], r["n_p"]) for name, rows in out.items() for r in rows if r["converged"]]
    best = min(conv) if conv else (None, None, None, None)
    return {"metric": "s to T = 1 (3D heat, Sec. 4.3 strong-scaling problem)", "value": best[0], "unit": "s",
            "form": "paper's uniform nodes: ISDC / IMLSDC / IPFASST over the whole interval (Table 1)",
            "best": {"config": best[1], "method": best[2], "n_p": best[3]}, "configs": out,
            "higher_is_better": False,
            "dtype": "f64", "data": "synthetic", "n_gpus": 1,
            "config": {"workload": "3D heat, nu=1/3, T=1, sin sin sin, uniform nodes: 127^3 3/2 (128 steps), "
                                   "127^3 5/3 (24 steps), 31^3 fourth-order stencil 5/3 (24 steps); rbgs V(2,2), "
                                   "2 V-cycles/solve, cubic interpolation between levels, "
                                   f"{a.table1_tol} residual 1e-9, F: {a.table1_f}"}}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the time-parallel "
              "multi-GPU path is not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import inputs
    from paper_1407_6486_amd import pfmg

    assert torch.cuda.is_available(), "no GPU visible"
    if a.form:
        fn = {"mixed": form_mixed, "batched": form_batched, "learned": form_learned, "nn-forward": form_nn_forward,
              "solve-policies": form_solve_policies, "heat1d": form_heat1d, "table1": form_table1,
              "weak3": form_weak3}[a.form]
        print(json.dumps(fn(pfmg, a), default=float), flush=True)
        return
    if a.cpu_full_block:
        u0_host, _ = inputs.random_fourier(a.n, 1407)
        print(json.dumps({"cpu_full_block": cpu_full_block(a.n, a.slices, u0_host), "host": host_info()}),
              flush=True)
        return
    if a.calibrate_copy:
        copy_calibration(pfmg)
    n, P = a.n, a.slices
    p = pfmg.pfmg_default_params(
        dim=3, n=n, n_slices=P, nu=1.0, dt=1e-3, vcycles_per_solve=a.vcycles,
        smoother=pfmg.SMOOTH_RBGS if a.smoother == "rbgs" else pfmg.SMOOTH_JACOBI,
        omega=1.0 if a.smoother == "rbgs" else 2.0 / 3.0,
        precision=pfmg.FP64 if a.precision == "fp64" else pfmg.MIXED, pfasst_tol=1e-10, pfasst_max_iter=a.max_iter)
    ctx = pfmg.Context(p)
    u0_host, _ = inputs.random_fourier(n, 1407)
    u0 = torch.from_numpy(u0_host).to("cuda")
    torch.cuda.synchronize()

    for _ in range(a.warmup):
        ctx.run_block(u0)
    torch.cuda.synchronize()

    # timed region: whole blocks as the library runs them (graph replays);
    # --steps 0 skips it (profiling runs of the event-timed blocks alone)
    v0 = ctx.vcycle_count(0)
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        st, it, res = ctx.run_block(u0)
        iters.append(it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fine_vcycles = (ctx.vcycle_count(0) - v0) / max(a.steps, 1)
    s_per_block = (t1 - t0) / a.steps if a.steps > 0 else None

    # dominant kernel: one more block with HIP events that each launch
    # stamps itself (hipExtLaunchKernel) on the stream it runs on (event
    # brackets run the block from the host, launch by launch).  Measured
    # twice: in a context whose coarse chain shares the main stream (the
    # sweeps run without the chain's kernels beside them, as under
    # rocprofv3, which serialises the two streams), and in the benchmark's
    # own context (the chain beside the sweeps)
    dominant = f"{a.smoother}@{n}"
    os.environ["PFMG_ONE_STREAM"] = "1"
    try:
        ctx1 = pfmg.Context(p)
    finally:
        del os.environ["PFMG_ONE_STREAM"]
    ctx1.run_block(u0)
    ctx1.timing_enable(dominant, True)
    ctx1.run_block(u0)
    launches, ms, nbytes = ctx1.timing_read()
    ctx1.timing_enable(None, False)
    ctx1.close()
    ctx.timing_enable(dominant, True)
    torch.cuda.synchronize()
    te0 = time.perf_counter()
    ctx.run_block(u0)
    torch.cuda.synchronize()
    eager_block_s = time.perf_counter() - te0
    launches_b, ms_b, nbytes_b = ctx.timing_read()
    ctx.timing_enable(None, False)

    # V-cycle throughput: one more block with every fine-grid V-cycle bracketed
    ctx.timing_enable(f"vcycle@{n}", True)
    ctx.run_block(u0)
    vl, vms, vbytes = ctx.timing_read()
    ctx.timing_enable(None, False)
    vcycle_gdofs = vbytes / (vms * 1e-3) / 1e9 if vms > 0 else None   # vbytes holds DOF x cycles

    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None
    tr = measured_traffic() if (n == 127 and P == 16 and a.smoother == "rbgs" and a.precision == "fp64") else None
    per_launch = nbytes / max(launches, 1)
    traffic = None
    if tr and abs(tr["algorithmic_bytes_per_launch"] - per_launch) <= 1e-6 * per_launch:
        traffic = round(tr["hbm_bytes_per_launch"])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic, "kernel": dominant, "launches": launches,
                "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2), "bytes_per_launch": per_launch,
                "avg_launch_us_beside_chain": round(ms_b * 1e3 / max(launches_b, 1), 2),
                "achieved_beside_chain": round(nbytes_b / (ms_b * 1e-3) / 1e9, 1) if ms_b > 0 else None,
                "eager_block_s": round(eager_block_s, 4),
                "copy_gbs": round(copy_bandwidth_gbs(pfmg), 1)}

    out = {
        "metric": "s to 1e-10 residual per PFASST block",
        "value": round(s_per_block, 5) if s_per_block else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(s_per_block * 1e3, 3) if s_per_block else None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"3D heat, {n}^3, {P} slices, dt=1e-3, Lobatto 5/3, "
                               f"{a.smoother} V(2,2), {a.vcycles} V-cycle(s)/solve, {a.precision}, seed 1407",
                   "n": n, "slices": P, "vcycles_per_solve": a.vcycles, "smoother": a.smoother,
                   "precision": a.precision, "parallelism": "single GPU, slices batched"},
        "iterations_per_block": iters,
        "final_residual": res if iters else None,
        "fine_vcycles_per_block": fine_vcycles,
        "vcycle_gdofs": round(vcycle_gdofs, 2) if vcycle_gdofs else None,
        "roofline": roofline,
    }
    if a.families:
        fams = {}
        for fam in ("rbgs", "resid_restrict", "prolong", "apply_L", "sdc_start", "sdc_rhs", "colloc_resid"):
            for g in (n, (n + 1) // 2 - 1):
                r = stamped_roofline(ctx, u0, fam, g)
                if r:
                    fams[r["kernel"]] = {k: r[k] for k in ("launches", "avg_launch_us", "bytes_per_launch",
                                                           "achieved")}
        out["families"] = fams
    if not a.no_cpu_baseline and iters:
        out["cpu_baseline"] = cpu_baseline(n, P, iters[-1], a.cpu_iters, u0_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
