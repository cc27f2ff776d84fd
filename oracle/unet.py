"""FP64 reference of the learned initial guess's network (TEST INFRASTRUCTURE
ONLY: used by the test suite, the smoke check and bench.py's CPU leg; the
product path never imports it).

The network predicts the correction of a node solve (I - alpha L_h) u = b
from its right-hand side and its plain initial guess U (the previous
iterate at the node, the guess the paper's inexact solves start from,
Sec. 2.3.1).  The correction e = u - U solves (I - alpha L_h) e = r with
r = b - (I - alpha L_h) U, so the inputs are made scale-free: per voxel
r / s, U / |U|_inf and alpha (n+1)^2, with s = |r|_inf; output y, guess
g = U + s y, training target (u - U) / s.

Architecture (a 3-level U-Net, base width 16): every convolution has 3^3
taps, a bias, and zero values outside the grid.  Levels follow the
multigrid grids: level l+1 has n_{l+1} = (n_l + 1) / 2 - 1 points per
dimension, coarse point J (1-based) sitting on fine point 2J.

    L0  conv  3 -> 16  relu          level 0
    L1  conv 16 -> 16  relu          level 0   -> skip s0
    L2  down 16 -> 32  relu          level 1   (out[J] = sum_d W[d] x[2J + d])
    L3  conv 32 -> 32  relu          level 1   -> skip s1
    L4  down 32 -> 64  relu          level 2
    L5  conv 64 -> 64  relu          level 2
    L6  conv 64 -> 64  relu          level 2
    L7  up   64 -> 32  relu          level 1   (out[i] = sum_{2J + d = i} W[d] x[J])
    L8  conv 64 -> 32  relu          level 1   input: concat(L7 out, s1)
    L9  conv 32 -> 32  relu          level 1
    L10 up   32 -> 16  relu          level 0
    L11 conv 32 -> 16  relu          level 0   input: concat(L10 out, s0)
    L12 conv 16 -> 16  relu          level 0
    L13 1x1  16 -> 1   (linear)      level 0

Weights W[co, ci, dz, dy, dx] (tap index d + 1 per axis), bias b[co].
Arrays are [channel, z, y, x] per sample, x fastest.  Loss: the mean of the
squared difference to the target over all voxels and samples.

Everything here is plain NumPy in float64; each convolution is a sum over
its 27 taps of channel contractions (einsum) on shifted views.
"""
from __future__ import annotations

import numpy as np

LAYERS = [
    # (kind, cin, cout, level_in, relu)
    ("conv", 3, 16, 0, True),
    ("conv", 16, 16, 0, True),
    ("down", 16, 32, 0, True),
    ("conv", 32, 32, 1, True),
    ("down", 32, 64, 1, True),
    ("conv", 64, 64, 2, True),
    ("conv", 64, 64, 2, True),
    ("up", 64, 32, 2, True),
    ("conv", 64, 32, 1, True),
    ("conv", 32, 32, 1, True),
    ("up", 32, 16, 1, True),
    ("conv", 32, 16, 0, True),
    ("conv", 16, 16, 0, True),
    ("pw", 16, 1, 0, False),
]


def coarser(n: int) -> int:
    return (n + 1) // 2 - 1


def taps(kind: str) -> int:
    return 1 if kind == "pw" else 27


def init_params(seed: int = 0):
    """He-normal weights, zero biases (the GPU trainer uses its own copy of
    this recipe; parity tests pass the same arrays to both)."""
    rng = np.random.default_rng(seed)
    params = []
    for kind, ci, co, _, _ in LAYERS:
        t = taps(kind)
        fan_in = ci * t
        shape = (co, ci, 3, 3, 3) if t == 27 else (co, ci, 1, 1, 1)
        w = rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)
        if kind == "pw":
            w *= 0.1
        params.append((w, np.zeros(co)))
    return params


# ------------------------------------------------------------ layer maps
def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))


def conv_same(x, w, b):
    """out[co, i] = b[co] + sum_ci sum_d w[co, ci, d] x[ci, i + d]."""
    ci, n = x.shape[0], x.shape[1]
    xp = _pad(x)
    out = np.zeros((w.shape[0], n, n, n)) + b[:, None, None, None]
    for a in range(3):
        for c in range(3):
            for e in range(3):
                out += np.einsum("oc,czyx->ozyx", w[:, :, a, c, e], xp[:, a:a + n, c:c + n, e:e + n])
    return out


def conv_down(x, w, b):
    """out[co, J] = b[co] + sum_ci sum_d w[co, ci, d] x[ci, 2J + d] (1-based J)."""
    n = x.shape[1]
    nc = coarser(n)
    xp = _pad(x)                      # padded index p holds 1-based point p
    out = np.zeros((w.shape[0], nc, nc, nc)) + b[:, None, None, None]
    for a in range(3):
        for c in range(3):
            for e in range(3):
                # 1-based 2J + d, J = 1..nc, d = a - 1 -> padded index 2J + a - 1
                sl = lambda t: slice(1 + t, 1 + t + 2 * nc, 2)
                out += np.einsum("oc,czyx->ozyx", w[:, :, a, c, e], xp[:, sl(a), sl(c), sl(e)])
    return out


def conv_up(x, w, b, n):
    """out[co, i] = b[co] + sum_ci sum_{J, d: 2J + d = i} w[co, ci, d] x[ci, J]
    on the fine grid of n points (x on the coarse grid (n+1)/2 - 1)."""
    nc = x.shape[1]
    outp = np.zeros((w.shape[0], n + 2, n + 2, n + 2))
    for a in range(3):
        for c in range(3):
            for e in range(3):
                sl = lambda t: slice(1 + t, 1 + t + 2 * nc, 2)
                outp[:, sl(a), sl(c), sl(e)] += np.einsum("oc,czyx->ozyx", w[:, :, a, c, e], x)
    return outp[:, 1:n + 1, 1:n + 1, 1:n + 1] + b[:, None, None, None]


def conv_pw(x, w, b):
    return np.einsum("oc,czyx->ozyx", w[:, :, 0, 0, 0], x) + b[:, None, None, None]


# --------------------------------------------------------- layer adjoints
def conv_same_bwd(x, w, dy):
    """Gradients of conv_same: (dx, dw, db)."""
    n = x.shape[1]
    xp = _pad(x)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(3):
        for c in range(3):
            for e in range(3):
                view = (slice(None), slice(a, a + n), slice(c, c + n), slice(e, e + n))
                dw[:, :, a, c, e] = np.einsum("ozyx,czyx->oc", dy, xp[view])
                dxp[view] += np.einsum("oc,ozyx->czyx", w[:, :, a, c, e], dy)
    return dxp[:, 1:n + 1, 1:n + 1, 1:n + 1], dw, dy.sum(axis=(1, 2, 3))


def conv_down_bwd(x, w, dy):
    n = x.shape[1]
    nc = dy.shape[1]
    xp = _pad(x)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(3):
        for c in range(3):
            for e in range(3):
                sl = lambda t: slice(1 + t, 1 + t + 2 * nc, 2)
                view = (slice(None), sl(a), sl(c), sl(e))
                dw[:, :, a, c, e] = np.einsum("ozyx,czyx->oc", dy, xp[view])
                dxp[view] += np.einsum("oc,ozyx->czyx", w[:, :, a, c, e], dy)
    return dxp[:, 1:n + 1, 1:n + 1, 1:n + 1], dw, dy.sum(axis=(1, 2, 3))


def conv_up_bwd(x, w, dy):
    nc = x.shape[1]
    dyp = _pad(dy)
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for a in range(3):
        for c in range(3):
            for e in range(3):
                sl = lambda t: slice(1 + t, 1 + t + 2 * nc, 2)
                view = dyp[:, sl(a), sl(c), sl(e)]
                dw[:, :, a, c, e] = np.einsum("ozyx,czyx->oc", view, x)
                dx += np.einsum("oc,ozyx->czyx", w[:, :, a, c, e], view)
    return dx, dw, dy.sum(axis=(1, 2, 3))


def conv_pw_bwd(x, w, dy):
    dx = np.einsum("oc,ozyx->czyx", w[:, :, 0, 0, 0], dy)
    dw = np.einsum("ozyx,czyx->oc", dy, x)[:, :, None, None, None]
    return dx, dw, dy.sum(axis=(1, 2, 3))


# ---------------------------------------------------------------- network
def forward(params, x):
    """x: [3, n, n, n] -> (y [1, n, n, n], cache of layer inputs/outputs)."""
    n0 = x.shape[1]
    acts = {}
    h = x
    cache = []
    skips = {}
    for i, ((kind, ci, co, lev, relu), (w, b)) in enumerate(zip(LAYERS, params)):
        if i == 8:
            h = np.concatenate([h, skips[1]], axis=0)
        if i == 11:
            h = np.concatenate([h, skips[0]], axis=0)
        inp = h
        if kind == "conv":
            z = conv_same(inp, w, b)
        elif kind == "down":
            z = conv_down(inp, w, b)
        elif kind == "up":
            n_out = n0 if lev == 1 else coarser(n0)
            z = conv_up(inp, w, b, n_out)
        else:
            z = conv_pw(inp, w, b)
        out = np.maximum(z, 0.0) if relu else z
        cache.append((inp, out))
        h = out
        if i == 1:
            skips[0] = out
        if i == 3:
            skips[1] = out
    acts["y"] = h
    return h, cache


def backward(params, cache, dy):
    """Gradient of <dy, y> with respect to every parameter and the input.
    Returns (grads [(dw, db)], dx)."""
    grads = [None] * len(LAYERS)
    dskip = {0: None, 1: None}
    g = dy
    for i in range(len(LAYERS) - 1, -1, -1):
        kind, ci, co, lev, relu = LAYERS[i]
        w, _ = params[i]
        inp, out = cache[i]
        if i == 1 and dskip[0] is not None:
            g = g + dskip[0]
        if i == 3 and dskip[1] is not None:
            g = g + dskip[1]
        dz = g * (out > 0) if relu else g
        if kind == "conv":
            dx, dw, db = conv_same_bwd(inp, w, dz)
        elif kind == "down":
            dx, dw, db = conv_down_bwd(inp, w, dz)
        elif kind == "up":
            dx, dw, db = conv_up_bwd(inp, w, dz)
        else:
            dx, dw, db = conv_pw_bwd(inp, w, dz)
        grads[i] = (dw, db)
        if i == 11:
            half = dx.shape[0] // 2
            dskip[0] = dx[half:]
            dx = dx[:half]
        if i == 8:
            half = dx.shape[0] // 2
            dskip[1] = dx[half:]
            dx = dx[:half]
        g = dx
    return grads, g


def loss_and_grads(params, xs, ts):
    """Mean squared error over a batch (lists of inputs and targets)."""
    total = 0.0
    count = sum(t.size for t in ts)
    acc = None
    for x, t in zip(xs, ts):
        y, cache = forward(params, x)
        r = y - t
        total += float(np.sum(r * r))
        grads, _ = backward(params, cache, 2.0 * r / count)
        if acc is None:
            acc = [(dw.copy(), db.copy()) for dw, db in grads]
        else:
            acc = [(a + dw, c + db) for (a, c), (dw, db) in zip(acc, grads)]
    return total / count, acc


def make_input(b, u, alpha):
    """Network input for the node solve (I - alpha L_h) u = b from the guess
    u: channels r / s, u / |u|_inf, alpha (n+1)^2 with r = b - (I - alpha L_h) u
    and s = |r|_inf (1 if zero).  Returns (x, s)."""
    from oracle import resid

    n = b.shape[0]
    r = resid(3, alpha, b, u)
    s = float(np.max(np.abs(r))) or 1.0
    su = float(np.max(np.abs(u))) or 1.0
    return np.stack([r / s, u / su, np.full(b.shape, alpha * (n + 1) ** 2)]), s


def guess(u, y, s):
    """Guess from the network output: g = u + s y."""
    return u + s * y
