/* C ABI of the learned warm start: a small 3D convolutional encoder-decoder
 * that maps a cell's density to its six periodic displacement fields, used as
 * the initial guess of the MG-PCG solve.  The network is not part of the
 * paper's method (which starts the solve from zero or from the previous
 * optimization iterate, Sec. 4.3); the plain cold-start solve stays the
 * fallback whenever the predicted field is not accurate enough.
 *
 * Every kernel is hand-written HIP for gfx950.  The 3x3x3 convolutions run on
 * the matrix cores (bf16 operands, FP32 accumulation) as implicit GEMMs; the
 * master parameters, the Adam moments, activations and gradients are FP32.
 *
 * Conventions
 *   Tensors are [batch][channel][z][y][x], x fastest, FP32, on the device of
 *   the handle's stream.  Convolutions are 3x3x3 with periodic (circular)
 *   padding, stride 1: y[b,o,v] = bias[o] + sum_{i,t} w[o,i,t] x[b,i,v+t],
 *   tap t = (dx+1) + 3 (dy+1) + 9 (dz+1) for offsets d in {-1,0,1}^3.
 *   Weights are [out][in][27].
 *   The caller owns every pointer argument; the library never frees them.
 *   Calls enqueue on the stream given at creation and return after enqueue,
 *   except those with host outputs, which synchronize.  Status codes are the
 *   hmg_status values of hmg.h.
 */
#ifndef HMG_NN_H
#define HMG_NN_H

#include <stdint.h>

#include "hmg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmg_nn_s* hmg_nn;

/* Architecture: `levels` resolution levels with base_channels * 2^l channels at
 * level l (two conv + ReLU per level and side, 2x average-pool down, nearest
 * 2x up, skip connections by channel concatenation), then a linear 3x3x3
 * output conv.  Defaults 4 / 8 / 1 / 18 give 368,712 weights + 370 biases. */
typedef struct hmg_nn_config {
  int32_t levels;         /* 1..5                                            */
  int32_t base_channels;  /* 1..32                                           */
  int32_t in_channels;    /* 1: the (filtered) density                       */
  int32_t out_channels;   /* 18: u / N for the six load cases x 3 components */
} hmg_nn_config;

/* Create a network with He-normal weights drawn from SplitMix64(seed) and zero
 * biases.  hip_stream: hipStream_t (NULL = default stream). */
hmg_status hmg_nn_create(const hmg_nn_config* cfg, void* hip_stream, uint64_t seed, hmg_nn* out);
hmg_status hmg_nn_destroy(hmg_nn net);

/* Number of FP32 parameters (weights of every layer in order, then biases). */
hmg_status hmg_nn_param_count(hmg_nn net, int64_t* count_out);
/* Copy the parameters / the accumulated gradients to or from host arrays of
 * param_count floats (synchronous). */
hmg_status hmg_nn_get_params(hmg_nn net, float* host, int64_t count);
hmg_status hmg_nn_set_params(hmg_nn net, const float* host, int64_t count);
hmg_status hmg_nn_get_grads(hmg_nn net, float* host, int64_t count);

/* y = net(x): x is [batch][in][dim^3], y is [batch][out][dim^3]; dim must be a
 * multiple of 2^(levels-1) and at least 2^(levels-1) * 2.  Keeps the
 * activations for hmg_nn_backward.  Work buffers grow to the largest
 * batch * dim^3 seen. */
hmg_status hmg_nn_forward(hmg_nn net, const float* x_dev, int32_t batch, int32_t dim,
                          float* y_dev);
/* Back-propagate dL/dy ([batch][out][dim^3], same shape as the last forward)
 * and ADD the parameter gradients to the accumulated ones. */
hmg_status hmg_nn_backward(hmg_nn net, const float* dy_dev);
hmg_status hmg_nn_zero_grad(hmg_nn net);
/* One Adam step (Kingma & Ba 2015) on the accumulated gradients; `step` is
 * the 1-based step number used for the bias corrections. */
hmg_status hmg_nn_adam_step(hmg_nn net, double lr, double beta1, double beta2, double eps,
                            int32_t step);
/* Mean squared error over `count` values: loss_out = mean((y - t)^2) (host,
 * synchronous), dy_dev = 2 (y - t) / count. */
hmg_status hmg_nn_mse(hmg_nn net, const float* y_dev, const float* t_dev, int64_t count,
                      float* dy_dev, double* loss_out);

/* Warm start of a solver context (cubic cells only): box-mean the density set
 * by hmg_set_density onto the multigrid level whose size is the largest of
 * N, N/2, ... not above 64 (and divisible by 2^(levels-1)), predict u / N
 * there, multiply by N, remove the per-component mean, prolongate to the fine
 * grid with the solver's trilinear P, scale each load case by its
 * energy-optimal factor alpha = u.f / u.K u (the scaled guess is never further
 * from the solution than zero in the energy norm), and apply one multigrid correction
 * u += M (f - K u) (a prediction that is right at low frequencies still
 * carries a large high-frequency residual on the fine grid, which one cycle
 * removes).  The result is kept as the iterate of the next
 * hmg_solve_cases(init = 1) when its relative residual ||f - K u|| / ||f||
 * (FP64, worst case over the six cases) is at most accept_relres; otherwise
 * the iterate is reset to zero (cold start).  relres_out receives that worst
 * relative residual, used_out 1 or 0. */
hmg_status hmg_warm_start(hmg_ctx ctx, hmg_nn net, double accept_relres, double* relres_out,
                          int32_t* used_out);

/* ---- single layers (used by the parity tests) ---------------------------
 * y = bias + conv(x, w) (then ReLU if relu != 0); y [B][Cout][D][H][W].     */
hmg_status hmg_conv3d_forward(void* hip_stream, const float* x, const float* w, const float* bias,
                              float* y, int32_t B, int32_t Cin, int32_t Cout, int32_t D,
                              int32_t H, int32_t W, int32_t relu);
/* dx += conv^T(dz, w): the adjoint of the convolution (bias excluded). */
hmg_status hmg_conv3d_backward_data(void* hip_stream, const float* dz, const float* w, float* dx,
                                    int32_t B, int32_t Cin, int32_t Cout, int32_t D, int32_t H,
                                    int32_t W);
/* dw += sum_{b,v} dz[b,o,v] x[b,i,v+t];  dbias += sum_{b,v} dz[b,o,v].
 * `work` must hold hmg_conv3d_workspace(B, Cin, Cout, D, H, W) floats. */
hmg_status hmg_conv3d_backward_weight(void* hip_stream, const float* x, const float* dz,
                                      float* dw, float* dbias, float* work, int32_t B,
                                      int32_t Cin, int32_t Cout, int32_t D, int32_t H, int32_t W);
int64_t hmg_conv3d_workspace(int32_t B, int32_t Cin, int32_t Cout, int32_t D, int32_t H,
                             int32_t W);

/* ---- allocation-free weight gradient -------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as hmg_conv3d_backward_weight (same kernels, same summation order),
 * with the partial sums held in a fixed 32 MiB array of the library on each
 * GPU instead of a workspace argument.  Calls no allocating routine.
 * Limit: hmg_conv3d_workspace(B, Cin, Cout, D, H, W) must not exceed
 * hmg_conv3d_noalloc_scratch_floats() (Cin * Cout <= 4854), else
 * HMG_E_INVALID.  Every call on one GPU uses that GPU's array: calls that
 * overlap on one GPU (other streams or host threads) race and must be
 * serialized by the caller.  dw and dbias accumulate as in the workspace form.
 * HMG_E_DEVICE if the array's device address cannot be looked up. */
hmg_status hmg_conv3d_backward_weight_noalloc(void* hip_stream, const float* x, const float* dz,
                                              float* dw, float* dbias, int32_t B, int32_t Cin,
                                              int32_t Cout, int32_t D, int32_t H, int32_t W);
int64_t hmg_conv3d_noalloc_scratch_floats(void);

#ifdef __cplusplus
}
#endif

#endif /* HMG_NN_H */
