"""Learned initial guess: network kernels against the FP64 network oracle,
the recording of training pairs, training, and the judged guess inside
PFASST.

Bars (BF16 activations and weights, FP32 accumulation):
  * per layer, from the GPU's own BF16 layer input: every output value
    within one BF16 unit (2^-8 relative) of the FP64 oracle, plus 1e-5 of
    the layer's largest value for FP32 accumulation order; the FP32 output
    layer to 1e-5;
  * per layer weight / bias gradients from the GPU's own input and
    upstream gradient: 2e-4 of the largest entry (FP32 sums over voxels);
    input gradients, as each producer layer stores the sum of its
    consumers' input gradients behind its ReLU mask: one BF16 unit of each
    addend and one of the sum;
  * end to end against the oracle in FP64 from the same BF16 parameters and
    inputs: output 3e-2 relative, loss 3e-2; per-layer gradients norm-wise
    within 0.25 with cosine >= 0.98 (the envelope of BF16 rounding of every
    intermediate over the forward and backward passes; the per-layer bars
    above are the parity of the kernels);
  * a recorded pair is consistent: (I - alpha L_h) target = r / |r| to BF16
    accuracy;
  * PFASST with the judged learned guess converges to the same collocation
    solution as the plain guess (1e-9).
"""
import sys

import numpy as np
import pytest

import inputs
import oracle as O
from oracle import unet as U
from tests import pins

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm device"
    from paper_1407_6486_amd import pfmg
    return pfmg


def to_bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in params])


def bf16_params(seed, bias_scale=0.05):
    rng = np.random.default_rng(seed + 100)
    ps = U.init_params(seed)
    return [(to_bf16(w), to_bf16(rng.standard_normal(b.shape) * bias_scale)) for w, b in ps]


def levels(n0):
    return [n0, U.coarser(n0), U.coarser(U.coarser(n0))]


def layer_io(i, n0):
    kind, ci, co, lev, _ = U.LAYERS[i]
    ns = levels(n0)
    lev_out = lev + 1 if kind == "down" else lev - 1 if kind == "up" else lev
    return ci, co, ns[lev], ns[lev_out]


def apply_layer(i, x, w, b, n_out):
    kind = U.LAYERS[i][0]
    if kind == "conv":
        return U.conv_same(x, w, b)
    if kind == "down":
        return U.conv_down(x, w, b)
    if kind == "up":
        return U.conv_up(x, w, b, n_out)
    return U.conv_pw(x, w, b)


def layer_bwd(i, x, w, dz):
    kind = U.LAYERS[i][0]
    return {"conv": U.conv_same_bwd, "down": U.conv_down_bwd, "up": U.conv_up_bwd, "pw": U.conv_pw_bwd}[kind](x, w, dz)


N0, B = 15, 2


def test_network_layers_match_oracle(pf):
    say(f"network forward per layer, n={N0}, batch {B}")
    params = bf16_params(1)
    rng = np.random.default_rng(2)
    x = to_bf16(rng.standard_normal((B, 3, N0, N0, N0)))
    net = pf.Net(N0, B, training=False)
    net.load(flat(params))
    y = net.forward(x.reshape(B, 3, -1))
    for i in range(13):
        ci, co, nin, nout = layer_io(i, N0)
        xin = net.tensor(i, 0, B, ci, nin)
        out = net.tensor(i, 1, B, co, nout)
        for s in range(B):
            want = np.maximum(apply_layer(i, xin[s], *params[i], nout), 0.0)
            tol = 2.0 ** -8 * np.abs(want) + 1e-5 * np.max(np.abs(want))
            bad = np.abs(out[s] - want) > tol
            assert not bad.any(), (i, s, float(np.max(np.abs(out[s] - want))), float(np.max(np.abs(want))))
    a8 = net.tensor(12, 1, B, 16, N0)
    for s in range(B):
        want = U.conv_pw(a8[s], *params[13])
        assert np.max(np.abs(y[s] - want.ravel())) <= 1e-5 * np.max(np.abs(want))
    # end to end against the oracle in FP64 from the same inputs
    for s in range(B):
        want, _ = U.forward(params, x[s])
        err = pins.rel_err(y[s], want.ravel())
        say(f"  sample {s}: output vs FP64 oracle {err:.2e}")
        assert err <= 3e-2
    net.close()


def test_network_gradients_match_oracle(pf):
    say(f"network backward per layer, n={N0}, batch {B}")
    params = bf16_params(3)
    rng = np.random.default_rng(4)
    x = to_bf16(rng.standard_normal((B, 3, N0, N0, N0)))
    t = rng.standard_normal((B, N0 ** 3)).astype(np.float32) * 0.3
    net = pf.Net(N0, B, training=True)
    net.load(flat(params))
    loss, g = net.gradients(x.reshape(B, 3, -1), t)
    # split the flat gradient per layer
    offs, o = [], 0
    for w, b in params:
        offs.append((o, o + w.size, o + w.size + b.size))
        o += w.size + b.size
    for i in range(13):
        ci, co, nin, nout = layer_io(i, N0)
        w = params[i][0]
        xin = net.tensor(i, 0, B, ci, nin)
        dz = net.tensor(i, 2, B, co, nout)
        dw = np.zeros_like(w)
        db = np.zeros(co)
        for s in range(B):
            _, dw_s, db_s = layer_bwd(i, xin[s], w, dz[s])
            dw += dw_s
            db += db_s
        gw = g[offs[i][0]:offs[i][1]].reshape(w.shape)
        gb = g[offs[i][1]:offs[i][2]]
        assert np.max(np.abs(gw - dw)) <= 2e-4 * np.max(np.abs(dw)) + 1e-12, (i, "w")
        assert np.max(np.abs(gb - db)) <= 2e-4 * np.max(np.abs(db)) + 1e-12, (i, "b")
    # input gradients: the upstream gradient each producer layer j stores
    # (after its ReLU mask) is the sum of its consumers' input gradients,
    # computed here in FP64 from the consumers' own GPU gradients
    consumers = {0: [(1, 0, 16)], 1: [(2, 0, 16), (11, 16, 32)], 2: [(3, 0, 32)], 3: [(4, 0, 32), (8, 32, 64)],
                 4: [(5, 0, 64)], 5: [(6, 0, 64)], 6: [(7, 0, 64)], 7: [(8, 0, 32)], 8: [(9, 0, 32)],
                 9: [(10, 0, 32)], 10: [(11, 0, 16)], 11: [(12, 0, 16)]}
    dxs = {}
    for i in range(1, 13):
        ci, co, nin, nout = layer_io(i, N0)
        dz = net.tensor(i, 2, B, co, nout)
        dxs[i] = [layer_bwd(i, np.zeros((ci,) + (nin,) * 3), params[i][0], dz[s])[0] for s in range(B)]
    for j, cons in consumers.items():
        _, co, _, nout = layer_io(j, N0)
        out = net.tensor(j, 1, B, co, nout)
        dz = net.tensor(j, 2, B, co, nout)
        for s in range(B):
            up = sum(dxs[i][s][a:b] for i, a, b in cons)
            mag = sum(np.abs(dxs[i][s][a:b]) for i, a, b in cons)
            want = np.where(out[s] > 0, up, 0.0)
            # each addend is rounded to BF16 before the sum, the sum once more
            tol = 2.0 ** -8 * (mag + np.abs(want)) + 1e-5 * np.max(np.abs(want))
            assert not (np.abs(dz[s] - want) > tol).any(), (j, s, float(np.max(np.abs(dz[s] - want))))
    # end to end: FP64 oracle gradients from the same parameters and inputs
    loss_o, grads_o = U.loss_and_grads(params, [x[s] for s in range(B)],
                                       [t[s].astype(np.float64).reshape(1, N0, N0, N0) for s in range(B)])
    assert abs(loss - loss_o) <= 3e-2 * loss_o
    go = flat(grads_o)
    stats = []
    for i in range(14):
        a, b_ = g[offs[i][0]:offs[i][2]], go[offs[i][0]:offs[i][2]]
        cos = float(np.dot(a, b_) / (np.linalg.norm(a) * np.linalg.norm(b_) + 1e-300))
        rel = float(np.linalg.norm(a - b_) / np.linalg.norm(b_))
        stats.append((rel, cos))
        say(f"  layer {i}: gradient vs FP64 oracle, norm-wise rel {rel:.2e}, cos {cos:.5f}")
    # BF16 rounding of every activation and upstream gradient over 26 layer
    # passes (and ReLU masks flipping near zero) against an all-FP64 network:
    # the gap grows from the output to the bottleneck (measured: norm-wise
    # <= 0.17, cosine >= 0.985 at 15^3 with random weights and targets); the
    # directions agree, as a wiring error would not let them
    for i, (rel, cos) in enumerate(stats):
        assert cos >= 0.98 and rel <= 0.25, (i, rel, cos)
    net.close()


def test_recorded_pairs_are_consistent_and_training_lowers_the_loss(pf):
    import torch

    n, P = 31, 4
    say(f"record pairs from full node solves, n={n}, P={P}; train")
    c = pf.Context(pf.pfmg_default_params(n=n, n_slices=P, nu=1.0, dt=2e-3, vcycles_per_solve=0, mg_tol=1e-10,
                                           pfasst_tol=1e-10, pfasst_max_iter=6))
    store = pf.PairStore(n, 400, P)
    store.attach(c)
    u0, _ = inputs.random_fourier(n, 77)
    c.run_block(u0)
    cnt = pf.pfmg_record_count(c.h)
    say(f"  recorded {cnt} pairs")
    assert cnt >= 6 * 4 * P
    pairs = store.pairs.float().cpu().numpy()
    ah2 = store.ah2.cpu().numpy()
    # consistency: (I - alpha L_h) target = r / |r|
    for k in (0, cnt // 2, cnt - 1):
        alpha = float(ah2[k]) / (n + 1) ** 2
        tgt = pairs[k, 2].reshape(n, n, n).astype(np.float64)
        r = pairs[k, 0].reshape(n, n, n).astype(np.float64)
        lhs = O.helm(3, alpha, tgt)
        assert np.max(np.abs(lhs - r)) <= 2e-2 * max(1.0, np.max(np.abs(r))), k
        assert abs(np.max(np.abs(r)) - 1.0) <= 1e-2
    net = pf.Net(n, 4, training=True)
    net.init(5)
    rng = np.random.default_rng(6)
    losses = []
    for step in range(120):
        idx = rng.integers(0, cnt, size=4)
        losses.append(net.train_step(store, idx, 2e-3))
    say(f"  loss first 10 {np.mean(losses[:10]):.3e} last 10 {np.mean(losses[-10:]):.3e}")
    assert np.isfinite(losses).all()
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])
    c.close()
    net.close()


def test_learned_guess_is_judged_and_converges(pf):
    n, P = 31, 4
    say(f"learned guess inside PFASST, n={n}, P={P}")
    kw = dict(n=n, n_slices=P, nu=1.0, dt=2e-3, vcycles_per_solve=0, mg_tol=1e-10, pfasst_tol=1e-10,
              pfasst_max_iter=200)
    # training data from other initial data
    rec = pf.Context(pf.pfmg_default_params(**kw))
    store = pf.PairStore(n, 2000, P)
    total = 0
    for seed in range(3):
        store.attach(rec, total)
        rec.run_block(inputs.random_fourier(n, 300 + seed)[0])
        total += pf.pfmg_record_count(rec.h)
        if total >= store.capacity - 200:
            break
    rec.close()
    net = pf.Net(n, P, training=True)
    net.init(7)
    rng = np.random.default_rng(8)
    for step in range(300):
        net.train_step(store, rng.integers(0, total, size=4), 2e-3 if step < 200 else 5e-4)
    u0, _ = inputs.random_fourier(n, 99)
    plain = pf.Context(pf.pfmg_default_params(**kw))
    st, it_p, res_p = plain.run_block(u0)
    learned = pf.Context(pf.pfmg_default_params(guess=pf.GUESS_LEARNED, **kw))
    pf.pfmg_attach_nn(learned.h, net.h)
    st2, it_l, res_l = learned.run_block(u0)
    tried, taken = pf.pfmg_guess_stats(learned.h)
    vp, vl = plain.vcycle_count(0), learned.vcycle_count(0)
    say(f"  plain: {it_p} iterations, {vp} fine V-cycles; learned: {it_l} iterations, {vl} fine V-cycles; "
        f"guess taken {taken} of {tried}")
    assert st == pf.OK and st2 == pf.OK and res_l <= 1e-10
    assert tried > 0 and 0 <= taken <= tried
    for p in range(P):
        assert pins.rel_err(learned.get(O.UF, p, 4), plain.get(O.UF, p, 4)) <= 1e-9
    # end to end against the closed form: at convergence every slice's end
    # value is sum_j a_j R44(dt nu mu_j)^(p+1) phi_j (Lobatto IIIA)
    g = pins.golden("lobatto_iiia.json")
    _, modes = inputs.random_fourier(n, 99)
    for p in range(P):
        want = np.zeros((n,) * 3)
        for a, k in zip(modes.amp, modes.k):
            want += a * pins.pade(2e-3 * pins.mu(n, k), g["pade44_num"]) ** (p + 1) * inputs.sine_mode(n, k, 3)
        assert pins.rel_err(learned.get(O.UF, p, 4), want) <= 1e-9, p
    plain.close()
    learned.close()
    net.close()
