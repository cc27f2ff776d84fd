"""Pins of the network oracle (oracle/unet.py) against definitions it does
not share code with: SciPy's correlation, brute-force loops, the adjoint
identity between the stride-2 and transposed convolutions, and central
finite differences of the whole network's loss."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import unet as U


def rand(rng, *shape):
    return rng.standard_normal(shape)


def test_conv_same_matches_scipy_correlation():
    rng = np.random.default_rng(1)
    x, w, b = rand(rng, 3, 7, 7, 7), rand(rng, 4, 3, 3, 3, 3), rand(rng, 4)
    want = np.zeros((4, 7, 7, 7))
    for o in range(4):
        want[o] = b[o] + sum(ndi.correlate(x[c], w[o, c], mode="constant", cval=0.0) for c in range(3))
    assert np.max(np.abs(U.conv_same(x, w, b) - want)) <= 1e-12


def test_down_is_same_conv_at_even_points():
    rng = np.random.default_rng(2)
    x, w, b = rand(rng, 2, 15, 15, 15), rand(rng, 3, 2, 3, 3, 3), rand(rng, 3)
    same = U.conv_same(x, w, b)
    # 1-based fine points 2J are 0-based indices 1, 3, ...
    assert np.max(np.abs(U.conv_down(x, w, b) - same[:, 1::2, 1::2, 1::2])) <= 1e-12


def test_up_matches_brute_force_scatter():
    rng = np.random.default_rng(3)
    nc, n = 3, 7
    x, w, b = rand(rng, 2, nc, nc, nc), rand(rng, 3, 2, 3, 3, 3), rand(rng, 3)
    want = np.zeros((3, n, n, n)) + b[:, None, None, None]
    for o in range(3):
        for c in range(2):
            for K in range(1, nc + 1):
                for J in range(1, nc + 1):
                    for I in range(1, nc + 1):
                        for dz in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dx in (-1, 0, 1):
                                    want[o, 2 * K + dz - 1, 2 * J + dy - 1, 2 * I + dx - 1] += \
                                        w[o, c, dz + 1, dy + 1, dx + 1] * x[c, K - 1, J - 1, I - 1]
    assert np.max(np.abs(U.conv_up(x, w, b, n) - want)) <= 1e-12


def test_up_is_adjoint_of_down():
    rng = np.random.default_rng(4)
    n, nc = 15, 7
    w = rand(rng, 5, 3, 3, 3, 3)
    x, y = rand(rng, 3, n, n, n), rand(rng, 5, nc, nc, nc)
    lhs = np.sum(U.conv_down(x, w, np.zeros(5)) * y)
    rhs = np.sum(x * U.conv_up(y, w.transpose(1, 0, 2, 3, 4), np.zeros(3), n))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_layer_gradients_are_adjoints():
    # <dy, L(x + t v)> linear in t: the input gradient of every layer map is
    # its adjoint, the weight gradient its derivative in w
    rng = np.random.default_rng(5)
    cases = [("conv", (2, 7, 7, 7), (3, 2, 3, 3, 3), None), ("down", (2, 7, 7, 7), (3, 2, 3, 3, 3), None),
             ("up", (2, 3, 3, 3), (3, 2, 3, 3, 3), 7), ("pw", (4, 5, 5, 5), (2, 4, 1, 1, 1), None)]
    fw = {"conv": U.conv_same, "down": U.conv_down, "pw": U.conv_pw}
    bw = {"conv": U.conv_same_bwd, "down": U.conv_down_bwd, "up": U.conv_up_bwd, "pw": U.conv_pw_bwd}
    for kind, xs, ws, n in cases:
        x, w, b = rand(rng, *xs), rand(rng, *ws), rand(rng, ws[0])
        f = (lambda x_, w_, b_: U.conv_up(x_, w_, b_, n)) if kind == "up" else fw[kind]
        y = f(x, w, b)
        dy = rand(rng, *y.shape)
        dx, dw, db = bw[kind](x, w, dy)
        vx, vw = rand(rng, *xs), rand(rng, *ws)
        zb = np.zeros_like(b)
        assert abs(np.sum(dy * f(vx, w, zb)) - np.sum(dx * vx)) <= 1e-10 * np.sum(np.abs(dx * vx))
        assert abs(np.sum(dy * f(x, vw, zb)) - np.sum(dw * vw)) <= 1e-10 * np.sum(np.abs(dw * vw))
        assert np.allclose(db, dy.sum(axis=(1, 2, 3)))


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(6)
    n = 7
    params = U.init_params(7)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    xs = [rand(rng, 3, n, n, n) for _ in range(2)]
    ts = [rand(rng, 1, n, n, n) for _ in range(2)]
    loss, grads = U.loss_and_grads(params, xs, ts)
    eps = 1e-6
    for li in range(len(U.LAYERS)):
        w, b = params[li]
        for which in ("w", "b"):
            arr = w if which == "w" else b
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp, _ = U.loss_and_grads(params, xs, ts)
                flat[idx] = old - eps
                lm, _ = U.loss_and_grads(params, xs, ts)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                an = (grads[li][0] if which == "w" else grads[li][1]).reshape(-1)[idx]
                assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (li, which, idx, fd, an)


def test_network_input_gradient_matches_finite_differences():
    rng = np.random.default_rng(8)
    n = 7
    params = U.init_params(9)
    x = rand(rng, 3, n, n, n)
    y, cache = U.forward(params, x)
    dy = rand(rng, *y.shape)
    _, dx = U.backward(params, cache, dy)
    eps = 1e-6
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (np.sum(dy * U.forward(params, xp)[0]) - np.sum(dy * U.forward(params, xm)[0])) / (2 * eps)
        assert abs(fd - dx[idx]) <= 1e-6 * max(abs(fd), 1e-3)


def test_input_channels_are_scale_free():
    import oracle as O

    rng = np.random.default_rng(10)
    n, alpha = 7, 0.01
    b, u = rng.standard_normal((n, n, n)), rng.standard_normal((n, n, n))
    x, s = U.make_input(b, u, alpha)
    r = b - O.helm(3, alpha, u)
    assert abs(s - np.max(np.abs(r))) <= 1e-15 * s and x.shape == (3, n, n, n)
    assert np.max(np.abs(x[0] - r / s)) <= 1e-15 and np.max(np.abs(x[1])) == 1.0
    assert np.all(x[2] == alpha * (n + 1) ** 2)
    # scaling the problem scales s, not the channels
    x2, s2 = U.make_input(3.0 * b, 3.0 * u, alpha)
    assert abs(s2 - 3.0 * s) <= 1e-14 * s and np.max(np.abs(x2 - x)) <= 1e-15
    # the exact correction is a zero-residual guess
    e = O.mg_solve(3, alpha, r, np.zeros_like(r), O.policy(cycles=0, tol=1e-14))[0]
    g = U.guess(u, e / s, s)
    assert np.max(np.abs(b - O.helm(3, alpha, g))) <= 1e-12 * np.max(np.abs(b))
