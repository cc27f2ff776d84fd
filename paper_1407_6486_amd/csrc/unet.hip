// The learned initial guess's network on the GPU (see unet.h).
#include <hip/hip_runtime.h>

#include <cstring>

#include "unet.h"

#define HC(x)                                  \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

namespace pfmg {
namespace {

constexpr int PW = 3;   // kind of the pointwise output layer

struct Spec {
    int kind, cin, cout, level;
};
const Spec SPEC[14] = {
    {nn::SAME, 3, 16, 0},  {nn::SAME, 16, 16, 0}, {nn::DOWN, 16, 32, 0}, {nn::SAME, 32, 32, 1},
    {nn::DOWN, 32, 64, 1}, {nn::SAME, 64, 64, 2}, {nn::SAME, 64, 64, 2}, {nn::UP, 64, 32, 2},
    {nn::SAME, 64, 32, 1}, {nn::SAME, 32, 32, 1}, {nn::UP, 32, 16, 1},   {nn::SAME, 32, 16, 0},
    {nn::SAME, 16, 16, 0}, {PW, 16, 1, 0}};

inline int cin8(int c) { return (c + 7) & ~7; }
inline nn::Act view(const nn::Act &a, int coff) { return nn::Act{a.p + coff, a.n, a.cs}; }
inline nn::Act none() { return nn::Act{nullptr, 0, 8}; }

}  // namespace

bool UNet::valid_n(int n0)
{
    // three levels, each odd and at least 3 points
    int n = n0;
    for (int l = 0; l < 3; ++l) {
        if (n < 3 || (n & 1) == 0) return false;
        n = (n + 1) / 2 - 1;
    }
    return true;
}

long UNet::param_count()
{
    long c = 0;
    for (const Spec &sp : SPEC) c += (sp.kind == PW ? 1L : 27L) * sp.cin * sp.cout + sp.cout;
    return c;
}

size_t UNet::carve(char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~(size_t)255;
        char *r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    n[1] = (n[0] + 1) / 2 - 1;
    n[2] = (n[1] + 1) / 2 - 1;
    nparams = param_count();
    params = (float *)take(nparams * 4);
    if (training) {
        grads = (float *)take(nparams * 4);
        m1 = (float *)take(nparams * 4);
        m2 = (float *)take(nparams * 4);
    }
    L.assign(14, UNetLayer{});
    long po = 0;
    for (int i = 0; i < 14; ++i) {
        const Spec &sp = SPEC[i];
        UNetLayer &l = L[i];
        l.kind = sp.kind;
        l.cin = sp.cin;
        l.cout = sp.cout;
        l.level = sp.level;
        l.w_off = po;
        po += (sp.kind == PW ? 1L : 27L) * sp.cin * sp.cout;
        l.b_off = po;
        po += sp.cout;
        if (sp.kind != PW) {
            l.wf = (nn::bf16 *)take(27L * sp.cout * cin8(sp.cin) * 2);
            if (training && i > 0) l.wb = (nn::bf16 *)take(27L * sp.cin * sp.cout * 2);
        }
    }
    auto act = [&](int lev, int cs) {
        const int nn_ = n[lev];
        return nn::Act{(nn::bf16 *)take((size_t)cap * nn::act_voxels(nn_) * cs * 2), nn_, cs};
    };
    x0 = act(0, 8);
    a0 = act(0, 16);
    c0 = act(0, 32);
    a1 = act(1, 32);
    c1 = act(1, 64);
    a2 = act(2, 64);
    a3 = act(2, 64);
    a4 = act(2, 64);
    a5 = act(1, 32);
    a6 = act(1, 32);
    a7 = act(0, 16);
    a8 = act(0, 16);
    y = (float *)take((size_t)cap * n[0] * n[0] * n[0] * 4);
    if (training) {
        target = (float *)take((size_t)cap * n[0] * n[0] * n[0] * 4);
        g_a8 = act(0, 16);
        g_a7 = act(0, 16);
        g_c0 = act(0, 32);
        g_a6 = act(1, 32);
        g_a5 = act(1, 32);
        g_c1 = act(1, 64);
        g_a4 = act(2, 64);
        g_a3 = act(2, 64);
        g_a2 = act(2, 64);
        g_s1 = act(1, 32);
        g_a1 = act(1, 32);
        g_s0 = act(0, 16);
        g_a0 = act(0, 16);
    }
    loss = (double *)take(8);
    idx = (int *)take((size_t)cap * 4);
    // forward tensors of every layer
    const nn::Act s0 = view(c0, 16), s1 = view(c1, 32);
    const nn::Act ins[14] = {x0, a0, s0, a1, s1, a2, a3, a4, c1, a5, a6, c0, a7, a8};
    const nn::Act outs[14] = {a0, s0, a1, s1, a2, a3, a4, view(c1, 0), a5, a6, view(c0, 0), a7, a8, none()};
    const nn::Act dins[14] = {none(), g_a0, g_s0, g_a1, g_s1, g_a2, g_a3, g_a4, g_c1, g_a5, g_a6, g_c0, g_a7, g_a8};
    const nn::Act douts[14] = {g_a0, g_s0, g_a1, g_s1, g_a2, g_a3, g_a4, view(g_c1, 0), g_a5, g_a6, view(g_c0, 0),
                               g_a7, g_a8, g_a8};
    for (int i = 0; i < 14; ++i) {
        L[i].in = ins[i];
        L[i].out = outs[i];
        L[i].din = dins[i];
        L[i].dout = douts[i];
    }
    ws_bytes = ((off + 255) & ~(size_t)255) + 256;
    return ws_bytes;
}

hipError_t UNet::refresh_weights()
{
    for (int i = 0; i < 13; ++i) {
        UNetLayer &l = L[i];
        HC(nn::weights_forward(params + l.w_off, l.cout, l.cin, cin8(l.cin), l.wf, s));
        if (l.wb) HC(nn::weights_backward(params + l.w_off, l.cout, l.cin, l.kind == nn::SAME, l.wb, s));
    }
    return hipSuccess;
}

hipError_t UNet::forward(int batch)
{
    if (batch < 1 || batch > cap) return hipErrorInvalidValue;
    for (int i = 0; i < 13; ++i) {
        const UNetLayer &l = L[i];
        HC(nn::conv((nn::Mode)l.kind, l.in, cin8(l.cin), l.out, l.cout, l.wf, params + l.b_off, true, batch, s));
    }
    return nn::pw_forward(a8, params + L[13].w_off, params + L[13].b_off, y, batch, s);
}

// Gradients of the mean squared error against `target`; count = the number
// of voxels the mean runs over.  Order: output layer, then every layer from
// the last: dZ = ReLU'(out) (dOut + skip gradient), weight and bias
// gradients from dZ and the layer input, then the input gradient (for the
// first layer none).
hipError_t UNet::backward(int batch, double count)
{
    if (!training || batch < 1 || batch > cap) return hipErrorInvalidValue;
    HC(nn::fill_f32(grads, 0.f, nparams, s));
    HC(hipMemsetAsync(loss, 0, 8, s));
    const UNetLayer &o = L[13];
    HC(nn::pw_loss_backward(a8, params + o.w_off, y, target, count, g_a8, grads + o.w_off, grads + o.b_off, loss,
                            batch, s));
    const nn::Act none_ = none();
    for (int i = 12; i >= 0; --i) {
        const UNetLayer &l = L[i];
        // skip gradients join the encoder outputs s0 (layer 1) and s1 (layer 3)
        const nn::Act skip = i == 1 ? view(g_c0, 16) : i == 3 ? view(g_c1, 32) : none_;
        HC(nn::relu_bwd(l.dout, skip, l.out, l.dout, l.cout, batch, s));
        HC(nn::conv_wgrad((nn::Mode)l.kind, l.in, l.cin, l.dout, l.cout, grads + l.w_off, batch, s));
        HC(nn::bias_grad(l.dout, l.cout, grads + l.b_off, batch, s));
        if (i == 0) break;
        const nn::Mode bm = l.kind == nn::SAME ? nn::SAME : l.kind == nn::DOWN ? nn::UP : nn::DOWN;
        HC(nn::conv(bm, l.dout, l.cout, l.din, l.cin, l.wb, nullptr, false, batch, s));
    }
    return hipSuccess;
}

hipError_t UNet::train_step(const nn::bf16 *pairs, const float *ah2, const int *idx_host, int batch, float lr,
                            double *loss_out)
{
    if (!training || batch < 1 || batch > cap) return hipErrorInvalidValue;
    HC(hipMemcpyAsync(idx, idx_host, sizeof(int) * batch, hipMemcpyHostToDevice, s));
    HC(nn::gather_batch(pairs, ah2, idx, batch, n[0], x0, target, s));
    HC(forward(batch));
    const double count = (double)batch * n[0] * n[0] * n[0];
    HC(backward(batch, count));
    HC(nn::adam(params, grads, m1, m2, nparams, lr, 0.9f, 0.999f, 1e-8f, ++adam_t, s));
    HC(refresh_weights());
    double l = 0;
    HC(hipMemcpyAsync(&l, loss, 8, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    if (loss_out) *loss_out = l / count;
    return hipSuccess;
}

hipError_t UNet::load_dense_input(const float *xd, int batch)
{
    if (batch < 1 || batch > cap) return hipErrorInvalidValue;
    return nn::load_input_dense(xd, batch, n[0], x0, s);
}

}  // namespace pfmg
