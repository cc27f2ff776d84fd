"""Training and evaluation of the learned initial guess through the C-ABI.

Pairs come from the validated solver itself: PFASST blocks on seeded
random-Fourier problems with full fine-level node solves record, for every
node solve, the scaled residual of the plain guess, the plain guess and the
scaled correction (pfmg_record).  The network trains on them with the
library's own forward, backward and Adam kernels (pfmg_nn_train_step), and
runs inside PFASST with guess = PFMG_GUESS_LEARNED, the FP64 residual
deciding per field whether its guess replaces the plain one.

    python -m paper_1407_6486_amd.learned --train-n 63 --pairs 20000 --steps 3000 --eval-n 127 --eval-slices 16
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def record(pf, n: int, pairs: int, slices: int = 4, first_run: int = 0, max_iter: int = 60, log=print):
    """Run seeded training problems until `pairs` node solves are recorded."""
    import inputs

    store = pf.PairStore(n, pairs, slices)
    total, r = 0, first_run
    t0 = time.perf_counter()
    while total < pairs - slices:
        u0, _, dt = inputs.training_problem(r, n)
        c = pf.Context(pf.pfmg_default_params(n=n, n_slices=slices, nu=1.0, dt=dt, vcycles_per_solve=0,
                                               mg_tol=1e-10, pfasst_tol=1e-10, pfasst_max_iter=max_iter))
        store.attach(c, total)
        c.run_block(u0)
        got = c.record_count()
        total += got
        log(f"  run {r}: dt {dt:.2e}, {got} pairs, {total} total, {time.perf_counter() - t0:.1f} s")
        c.close()
        r += 1
    return store, total


def train(pf, store, count: int, steps: int, batch: int = 8, lr: float = 2e-3, seed: int = 0, log=print):
    net = pf.Net(store.n, batch, training=True)
    net.init(seed)
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.perf_counter()
    for k in range(steps):
        # cosine decay to a tenth of the initial rate
        rate = lr * (0.1 + 0.45 * (1 + np.cos(np.pi * k / max(1, steps))))
        losses.append(net.train_step(store, rng.integers(0, count, size=batch), float(rate), n_pairs=count))
        if (k + 1) % max(1, steps // 10) == 0:
            log(f"  step {k + 1}: loss {np.mean(losses[-50:]):.3e}  {time.perf_counter() - t0:.1f} s")
    return net, losses, time.perf_counter() - t0


def evaluate(pf, params, n: int, slices: int, thresholds=(0.0,), seed: int = 1407, mg_tol: float = 1e-12,
             log=print):
    """One block of the 127^3 random-Fourier problem (seed 1407) with full node solves (to mg_tol),
    plain guess against the learned guess offered to solves whose plain
    guess has relative residual above each threshold."""
    import torch

    import inputs

    u0, _ = inputs.random_fourier(n, seed)
    kw = dict(n=n, n_slices=slices, nu=1.0, dt=1e-3, vcycles_per_solve=0, mg_tol=mg_tol, pfasst_tol=1e-10,
              pfasst_max_iter=400)
    out = {}
    net = pf.Net(n, slices, training=False)
    net.load(params)
    ref = None
    for mode in ["plain"] + [f"learned@{t:g}" for t in thresholds]:
        learned = mode != "plain"
        extra = dict(guess=pf.GUESS_LEARNED, guess_min_relres=float(mode.split("@")[1])) if learned else {}
        c = pf.Context(pf.pfmg_default_params(**kw, **extra))
        if learned:
            c.attach_nn(net)
        c.run_block(u0)                       # warm-up (tuning, first-touch)
        v0 = c.vcycle_count(0), c.vcycle_count(1)
        g0 = c.guess_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, res = c.run_block(u0)
        torch.cuda.synchronize()
        dt_block = time.perf_counter() - t0
        g1 = c.guess_stats()
        end = [c.get(0, p, 4) for p in (0, slices - 1)]
        if ref is None:
            ref = end
        diff = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b))) for a, b in zip(end, ref))
        out[mode] = {"s_per_block": dt_block, "iterations": it, "residual": res, "status": st,
                     "fine_vcycles": c.vcycle_count(0) - v0[0], "coarse_vcycles": c.vcycle_count(1) - v0[1],
                     "guesses_offered": g1[0] - g0[0], "guesses_taken": g1[1] - g0[1], "end_state_rel_diff": diff}
        log(f"  {mode}: {dt_block:.3f} s, {it} iterations, residual {res:.2e}, fine V-cycles "
            f"{out[mode]['fine_vcycles']}, guess taken {out[mode]['guesses_taken']} of "
            f"{out[mode]['guesses_offered']}, end state vs plain {diff:.1e}")
        c.close()
    net.close()
    return out


def inference_time(pf, params, n: int, batch: int, reps: int = 5):
    """Seconds per forward pass of `batch` samples of n^3 (device data)."""
    import torch

    net = pf.Net(n, batch, training=False)
    net.load(params)
    x = torch.zeros((batch, 3, n ** 3), dtype=torch.float32, device="cuda")
    y = torch.empty((batch, n ** 3), dtype=torch.float32, device="cuda")
    pf.pfmg_nn_forward(net.h, x.data_ptr(), batch, y.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pf.pfmg_nn_forward(net.h, x.data_ptr(), batch, y.data_ptr())
    torch.cuda.synchronize()
    net.close()
    return (time.perf_counter() - t0) / reps


def flops_per_voxel() -> float:
    """Multiply-adds x 2 of one forward pass per fine voxel (the coarse
    levels hold 1/8 and 1/64 of the voxels; the transposed convolutions
    apply 27/8 taps per output voxel on average)."""
    taps = {0: 1.0, 1: 1 / 8, 2: 1 / 64}
    spec = [(27, 3, 16, 0), (27, 16, 16, 0), (27, 16, 32, 1), (27, 32, 32, 1), (27, 32, 64, 2), (27, 64, 64, 2),
            (27, 64, 64, 2), (27 / 8, 64, 32, 1), (27, 64, 32, 1), (27, 32, 32, 1), (27 / 8, 32, 16, 0),
            (27, 32, 16, 0), (27, 16, 16, 0), (1, 16, 1, 0)]
    return 2.0 * sum(t * ci * co * taps[lev] for t, ci, co, lev in spec)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-n", type=int, default=63)
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-n", type=int, default=127)
    ap.add_argument("--eval-slices", type=int, default=16)
    ap.add_argument("--thresholds", default="0,1e-6,1e-4",
                    help="guess_min_relres values to evaluate (comma-separated)")
    ap.add_argument("--mg-tol", type=float, default=1e-12, help="per-solve relative tolerance")
    ap.add_argument("--save", default=None, help="write the trained parameters (.npy)")
    a = ap.parse_args()
    from paper_1407_6486_amd import pfmg as pf

    log = lambda m: print(m, flush=True)
    log(f"recording {a.pairs} pairs at {a.train_n}^3")
    t0 = time.perf_counter()
    store, count = record(pf, a.train_n, a.pairs, log=log)
    t_rec = time.perf_counter() - t0
    log(f"training {a.steps} steps, batch {a.batch}")
    net, losses, t_train = train(pf, store, count, a.steps, a.batch, a.lr, log=log)
    params = net.save()
    net.close()
    if a.save:
        np.save(a.save, params)
    t_inf = inference_time(pf, params, a.eval_n, a.eval_slices)
    fl = flops_per_voxel() * a.eval_n ** 3 * a.eval_slices
    log(f"inference {a.eval_slices} x {a.eval_n}^3: {t_inf * 1e3:.2f} ms, {fl / t_inf / 1e12:.1f} TFLOP/s")
    log(f"evaluating at {a.eval_n}^3, {a.eval_slices} slices")
    ev = evaluate(pf, params, a.eval_n, a.eval_slices, [float(t) for t in a.thresholds.split(",")],
                  mg_tol=a.mg_tol, log=log)
    print(json.dumps({"pairs": count, "record_s": round(t_rec, 1), "train_steps": a.steps, "train_s": round(t_train, 1),
                      "loss_first": float(np.mean(losses[:50])), "loss_last": float(np.mean(losses[-50:])),
                      "inference_ms": round(t_inf * 1e3, 3), "inference_tflops": round(fl / t_inf / 1e12, 2),
                      "eval": ev}), flush=True)


if __name__ == "__main__":
    main()
