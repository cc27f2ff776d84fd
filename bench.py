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
launches bracketed by HIP events on the stream they run on during one more
block of the same workload; HBM traffic from the committed counter summary
while the kernel source and launch shape are unchanged) and the oracle
timed on the host.
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
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain copy of known size three times (reference for HBM counters)")
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


CALIB_N = 255


def copy_calibration(pfmg):
    """A plain copy of known size for the HBM counters: the library's pack
    kernel (one load and one store per point) gathers one 255^3 field into a
    dense array, three times.  Reads: 255^2 rows of 2048 bytes (each row's
    255 values plus its halo word share 16 whole 128-byte lines); writes:
    255^3 x 8 bytes."""
    import torch

    c = pfmg.Context(pfmg.pfmg_default_params(dim=3, n=CALIB_N, n_slices=1, nodes_coarse=0))
    out = torch.empty((CALIB_N,) * 3, dtype=torch.float64, device="cuda")
    for _ in range(3):
        pfmg.pfmg_get(c.h, pfmg.U_FINE, 0, 0, out.data_ptr(), True)
    torch.cuda.synchronize()
    c.close()


def cpu_baseline(n, P, iters_gpu, cpu_iters, u0):
    """The oracle as it stands, on the host: predictor + cpu_iters iterations,
    extrapolated to the iteration count of the block."""
    import oracle as O

    t0 = time.perf_counter()
    orc = O.Pfasst(3, n, 1.0, 1e-3, P, 5, 3, O.policy(cycles=1))
    orc.set_initial(u0)
    t1 = time.perf_counter()
    for _ in range(cpu_iters):
        orc.iterate()
    t2 = time.perf_counter()
    per_iter = (t2 - t1) / cpu_iters
    est = (t1 - t0) + per_iter * iters_gpu
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(est, 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"predictor ({t1 - t0:.2f} s) + {cpu_iters} iterations ({per_iter:.2f} s each) of the "
                      f"same block on the host, extrapolated to the {iters_gpu} iterations the block needs"}


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

    # timed region: whole blocks as the library runs them (graph replays)
    v0 = ctx.vcycle_count(0)
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        st, it, res = ctx.run_block(u0)
        iters.append(it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fine_vcycles = (ctx.vcycle_count(0) - v0) / a.steps
    s_per_block = (t1 - t0) / a.steps

    # dominant kernel: one more block with HIP events around each of its
    # launches on the stream it runs on (event brackets run the block from
    # the host, launch by launch)
    dominant = f"{a.smoother}@{n}"
    ctx.timing_enable(dominant, True)
    ctx.run_block(u0)
    launches, ms, nbytes = ctx.timing_read()
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
        traffic = tr["hbm_bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic, "kernel": dominant, "launches": launches,
                "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2), "bytes_per_launch": per_launch}

    out = {
        "metric": "s to 1e-10 residual per PFASST block",
        "value": round(s_per_block, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(s_per_block * 1e3, 3),
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
        "final_residual": res,
        "fine_vcycles_per_block": fine_vcycles,
        "vcycle_gdofs": round(vcycle_gdofs, 2) if vcycle_gdofs else None,
        "roofline": roofline,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, P, iters[-1], a.cpu_iters, u0_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
