// The learned initial guess's network on the GPU: a 3-level U-Net (widths
// 16/32/64) on the multigrid grids n0 -> n1 = (n0+1)/2 - 1 -> n2, BF16
// activations and weights, FP32 accumulation, FP32 master weights, Adam.
//
//   L0  conv  3 -> 16      x0 -> a0
//   L1  conv 16 -> 16      a0 -> c0[16:32]   (skip s0)
//   L2  down 16 -> 32      s0 -> a1
//   L3  conv 32 -> 32      a1 -> c1[32:64]   (skip s1)
//   L4  down 32 -> 64      s1 -> a2
//   L5  conv 64 -> 64      a2 -> a3
//   L6  conv 64 -> 64      a3 -> a4
//   L7  up   64 -> 32      a4 -> c1[0:32]
//   L8  conv 64 -> 32      c1 -> a5
//   L9  conv 32 -> 32      a5 -> a6
//   L10 up   32 -> 16      a6 -> c0[0:16]
//   L11 conv 32 -> 16      c0 -> a7
//   L12 conv 16 -> 16      a7 -> a8
//   L13 1x1  16 -> 1       a8 -> y  (FP32, linear)
// All but L13 apply a ReLU.  Parameters: per layer W [27][cout][cin] then
// b [cout] (L13: w [16], b [1]), concatenated in layer order.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "nn.h"

namespace pfmg {

struct UNetLayer {
    int kind;       // nn::SAME / DOWN / UP, or 3 for the pointwise output
    int cin, cout, level;
    long w_off, b_off;              // offsets in the parameter array
    nn::bf16 *wf = nullptr;         // forward weights [27][cout][cin8]
    nn::bf16 *wb = nullptr;         // backward-data weights [27][cin][cout]
    nn::Act in, out;                // forward tensors
    nn::Act din, dout;              // gradient tensors (din: of the input)
};

struct UNet {
    int n[3] = {0, 0, 0};
    int cap = 0;                    // samples per batch
    bool training = false;
    hipStream_t s = nullptr;
    std::vector<UNetLayer> L;
    long nparams = 0;
    float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
    nn::Act x0{}, a0{}, c0{}, a1{}, c1{}, a2{}, a3{}, a4{}, a5{}, a6{}, a7{}, a8{};
    nn::Act g_a8{}, g_a7{}, g_c0{}, g_a6{}, g_a5{}, g_c1{}, g_a4{}, g_a3{}, g_a2{}, g_s1{}, g_a1{}, g_s0{}, g_a0{};
    float *y = nullptr, *target = nullptr;
    double *loss = nullptr;
    int *idx = nullptr;
    int adam_t = 0;
    size_t ws_bytes = 0;

    static bool valid_n(int n0);
    // Lay out the workspace (base == nullptr: size only).
    size_t carve(char *base);
    static long param_count();
    hipError_t refresh_weights();                  // masters -> BF16 layouts
    hipError_t forward(int batch);                 // x0 -> y
    hipError_t backward(int batch, double count);  // loss and gradients (grads zeroed here)
    hipError_t train_step(const nn::bf16 *pairs, const float *ah2, const int *idx_host, int batch, float lr,
                          double *loss_out);
    hipError_t load_dense_input(const float *xd, int batch);   // [batch][3][n^3] FP32 -> x0
};

}  // namespace pfmg
