// Kernels of the learned initial guess's network: 3D convolutions in BF16 on
// MFMA with FP32 accumulation, their backward passes, and the elementwise
// and data-movement kernels around them.
//
// Activations are BF16, channels-last, with a one-voxel zero halo: element
// (sample s, z, y, x, channel c), z/y/x in 0..n+1, sits at
//     p[(((s (n+2) + z) (n+2) + y) (n+2) + x) cs + c]
// where p already includes the tensor's channel offset inside a wider
// buffer (the skip concatenations share one buffer: the decoder's
// upsampled tensor in the first channels, the encoder's skip in the rest).
// Halos are zeroed once and never written.
//
// Convolution modes (grids follow the multigrid hierarchy, coarse point J
// on fine point 2J, 1-based):
//   SAME  out[i] = sum_d W[d] x[i + d]                      (3^3 taps)
//   DOWN  out[J] = sum_d W[d] x[2J + d]                     (fine -> coarse)
//   UP    out[i] = sum_{J, d : 2J + d = i} W[d] x[J]        (coarse -> fine)
// UP runs per parity class of the output point (per axis: even i takes
// d = 0, odd i takes d = +1 and d = -1), so no work is spent on zero taps.
// The backward pass of SAME is SAME with transposed, tap-flipped weights;
// that of DOWN is UP and that of UP is DOWN, with transposed weights.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.h"
#include "tile.h"

namespace pfmg {
namespace nn {

typedef __bf16 bf16;

struct Act {
    bf16 *p;     // sample 0, voxel (0,0,0), first channel of the tensor
    int n;       // interior points per axis
    int cs;      // channel stride of the buffer (multiple of 8)
};

inline long act_voxels(int n) { return (long)(n + 2) * (n + 2) * (n + 2); }

enum Mode { SAME = 0, DOWN = 1, UP = 2 };

// out = act(conv(in) + bias).  cin: input channels read (a multiple of 8
// after padding: channels cin..cin8-1 of the weights are zero); cout a
// multiple of 16.  W: BF16 [27][cout][cin8] (tap = (dz+1) 9 + (dy+1) 3 +
// (dx+1)); bias FP32 [cout] or nullptr; relu applies max(., 0).
hipError_t conv(Mode mode, const Act &in, int cin8, const Act &out, int cout, const bf16 *W, const float *bias,
                bool relu, int batch, hipStream_t s);

// dW[tap][co][ci] += sum over the layer's voxels of dZ[co] x[ci] at the
// tap's pair of points (FP32 accumulation, atomics).  cin: input channels.
hipError_t conv_wgrad(Mode mode, const Act &x, int cin, const Act &dz, int cout, float *dW, int batch,
                      hipStream_t s);
// db[c] += sum over voxels of dz[c]
hipError_t bias_grad(const Act &dz, int cout, float *db, int batch, hipStream_t s);
// dz = (dy + dskip) * (y > 0) on interior voxels (dskip may be null; dz may
// alias dy)
hipError_t relu_bwd(const Act &dy, const Act &dskip, const Act &y, const Act &dz, int c, int batch, hipStream_t s);

// Pointwise output layer (16 -> 1): y = w . x + b, FP32 dense [batch][n^3].
hipError_t pw_forward(const Act &x, const float *w, const float *b, float *y, int batch, hipStream_t s);
// Loss and its backward: with r = y - t, loss_acc[0] += sum r^2; dx = (2 r /
// count) w (BF16); dw[c] += sum (2 r / count) x_c; db += sum 2 r / count.
hipError_t pw_loss_backward(const Act &x, const float *w, const float *y, const float *t, double count,
                            const Act &dx, float *dw, float *db, double *loss_acc, int batch, hipStream_t s);

// Weight layouts from FP32 masters [27][cout][cin] (kernel layout):
//   forward  BF16 [27][cout][cin8]
//   backward BF16 [27][cin][cout] (transposed; SAME also flips the taps)
hipError_t weights_forward(const float *Wm, int cout, int cin, int cin8, bf16 *Wf, hipStream_t s);
hipError_t weights_backward(const float *Wm, int cout, int cin, bool flip, bf16 *Wb, hipStream_t s);

// Adam on a flat FP32 parameter array (bias-corrected, step t >= 1).
hipError_t adam(float *p, const float *g, float *m, float *v, long count, float lr, float beta1, float beta2,
                float eps, int t, hipStream_t s);
hipError_t fill_f32(float *p, float v, long count, hipStream_t s);

// ---- data movement between the solver's fields and the network
// Network input for the node solves of `t` (one sample per field):
// x0[0] = r / sr, x0[1] = u / su, x0[2] = alpha (n+1)^2, x0[3..7] = 0, with
// r = b - (I - alpha L_h) u; alpha per field from t's scalar table (or
// `alpha`), sr / su per field (device).
hipError_t make_input(const Tiling &t, double alpha, View<double> b, View<double> u, const double *sr,
                      const double *su, const Act &x0, hipStream_t s);
// g = u + sr y  (y FP32 dense per field) written to `g`.
hipError_t apply_guess(const Tiling &t, View<double> u, const float *y, const double *sr, View<double> g,
                       hipStream_t s);
// dense FP32 [batch][c][n^3] copy of a tensor's c channels (tests, inspection)
hipError_t act_to_dense(const Act &a, int c, int batch, float *dst, hipStream_t s);
// x0 from dense FP32 inputs [batch][3][n^3] (channels 3..7 zero).
hipError_t load_input_dense(const float *xd, int batch, int n, const Act &x0, hipStream_t s);
// Training batch from a pair store: sample q takes pair idx[q]; pairs hold
// BF16 dense [pair][3][n^3] (r / sr, u / su, target) and FP32 alpha (n+1)^2.
hipError_t gather_batch(const bf16 *pairs, const float *ah2, const int *idx, int batch, int n, const Act &x0,
                        float *target, hipStream_t s);
// Record one node solve per field into pairs[slot0 + field] (channels 0, 1
// before the solve; the target after it, from the saved guess `u0`):
hipError_t record_inputs(const Tiling &t, double alpha, View<double> b, View<double> u, const double *sr,
                         const double *su, bf16 *pairs, float *ah2, long slot0, double *u0, hipStream_t s);
hipError_t record_target(const Tiling &t, View<double> u, const double *sr, const double *u0, bf16 *pairs,
                         long slot0, hipStream_t s);

}  // namespace nn
}  // namespace pfmg
