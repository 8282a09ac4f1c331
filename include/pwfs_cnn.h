/*
 * pwfs_cnn.h -- C ABI of the learned modal reconstructor (CNN) of the
 * pyramid sensor library.
 *
 * The network replaces or backs up the modal reconstructor of the paper's
 * sensor chain (Sec. 4, Tab. 1 "modalrec", Tab. 2 rec.in_slopes ->
 * out_modes): it maps the four binned pupil images to modal (KL)
 * coefficients that feed the same integrator.  The paper has no learned
 * part; the architecture is fixed by this library:
 *   input  [B][S][S][4] float (NHWC), from pwfs_cnn_prepare
 *   conv 3x3 stride 2 pad 1, 4 -> c1, ReLU; conv c1 -> c2, ReLU; conv c2 -> c3, ReLU
 *   flatten in (y, x, channel) order; fully connected -> hidden, ReLU; -> n_out
 * Parameters are one flat FP32 vector: w1 [c1][4][3][3], b1 [c1],
 * w2 [c2][c1][3][3], b2, w3 [c3][c2][3][3], b3, fw1 [hidden][flat], fb1,
 * fw2 [n_out][hidden], fb2 (C order).  Products run on bf16 MFMA with FP32
 * accumulation (weights and activations rounded to bf16 as GEMM operands);
 * biases, loss, gradients, Adam moments and master weights are FP32.
 * Loss: mean over all outputs of w_b (prediction - target)^2, with an optional
 * weight w_b per frame (1 when no weights are given).
 *
 * Memory and errors follow pwfs.h: "device" pointers are caller-owned
 * allocations on the device current at create time; calls are
 * asynchronous on `stream`; argument errors are reported before launch;
 * there is no CPU fallback.
 */
#ifndef PWFS_CNN_H
#define PWFS_CNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pwfs_cnn_s* pwfs_cnn_t;

typedef struct {
  int32_t n_sub;      /* S: input side (40 at the LBT-like geometry), 4 <= S <= 256 */
  int32_t c1, c2, c3; /* conv channels (32, 64, 64), each 1..256                    */
  int32_t hidden;     /* hidden width (2048), 1..16384                              */
  int32_t n_out;      /* outputs (600 modes), 1..16384                              */
  int32_t batch_max;  /* activation workspace size in frames, 1..65535              */
  int32_t reserved;   /* must be 0                                                  */
} pwfs_cnn_config_t;

/* Allocate parameters (zero), Adam state and workspace for batch_max frames. */
int pwfs_cnn_create(const pwfs_cnn_config_t* cfg, pwfs_cnn_t* out);

/* Number of parameters (length of the flat vector). */
int pwfs_cnn_num_params(pwfs_cnn_t net, int64_t* n_params);

/* Load the flat FP32 parameter vector from device memory and reset the
 * Adam moments and step count. */
int pwfs_cnn_set_params(pwfs_cnn_t net, const float* d_params, void* stream);

/* Copy the flat FP32 master parameters into device memory. */
int pwfs_cnn_get_params(pwfs_cnn_t net, float* d_params, void* stream);

/* Optimiser state, for checkpoints: the Adam moments m and v (flat FP32,
 * the parameters' order, device memory, n_params each) and the step count
 * (Adam's bias correction uses it).  A checkpoint is the parameters
 * (pwfs_cnn_get_params) and this state; restoring is pwfs_cnn_set_params
 * (which resets the state) followed by pwfs_cnn_set_optimizer, after which
 * training continues exactly as if it had never stopped.  Stream-ordered
 * copies; PWFS_ERR_INVALID_ARG for NULL pointers or a negative step. */
int pwfs_cnn_get_optimizer(pwfs_cnn_t net, float* d_m, float* d_v, int64_t* step, void* stream);
int pwfs_cnn_set_optimizer(pwfs_cnn_t net, const float* d_m, const float* d_v, int64_t step, void* stream);

/* Network input from binned pupils.
 *   d_pupils [B][4][S][S], d_ref_pupils [4][S][S] (flat-wavefront pupils),
 *   d_valid [n_valid] int32 subaperture indices j = iy * S + ix.
 *   d_x [B][S][S][4] = pupils / n - ref / n_ref on valid subapertures, 0
 *   elsewhere, with n (n_ref) the mean total flux over valid subapertures
 *   of the frame (of the reference). */
int pwfs_cnn_prepare(const float* d_pupils, const float* d_ref_pupils, const int32_t* d_valid,
                     int32_t n_valid, int32_t B, int32_t S, float* d_x, void* stream);

/* Inference: d_out [B][n_out] from d_x [B][S][S][4].  B <= batch_max. */
int pwfs_cnn_forward(pwfs_cnn_t net, const float* d_x, int32_t B, float* d_out, void* stream);

/* Inference accumulated into d_out: d_out = alpha * net(d_x) + beta * d_out
 * (an integrator step of the learned reconstructor is alpha = gain,
 * beta = 1).  d_out is read when beta != 0. */
int pwfs_cnn_forward_acc(pwfs_cnn_t net, const float* d_x, int32_t B, float alpha, float beta, float* d_out,
                         void* stream);

/* Loss and parameter gradients (flat FP32, same order as the parameters)
 * for targets d_target [B][n_out] and per-frame weights d_weights [B] (NULL:
 * all 1); d_loss (1 float) and d_grads may be NULL.
 * The backward pass (also in pwfs_cnn_train_step) runs the loss sum and the
 * weight gradients of all layers but the first on a second stream of the
 * network (default priority) beside the chain of data gradients on `stream`
 * (which ends with the first layer's weight gradient), forked from and joined back into `stream` with
 * events: the call as a whole is ordered after earlier work on `stream` and
 * before later work on it, and a graph capture of `stream` takes in both.
 * Calls on one network must not overlap. */
int pwfs_cnn_gradients(pwfs_cnn_t net, const float* d_x, const float* d_target, const float* d_weights,
                       int32_t B, float* d_grads, float* d_loss, void* stream);

/* One training step (weights as in pwfs_cnn_gradients): forward, MSE loss, backward, Adam update of the FP32
 * master weights (step count incremented), bf16 weight copies refreshed.  The step count and Adam's bias
 * corrections are host state passed to the kernels: a captured graph of this call replays the step count
 * it was captured with.  The Adam update of every parameter but the first layer's runs on the network's
 * second stream (once the chain has read those weights for the last time), joined back into `stream`
 * before the call returns, like the backward pass's weight gradients.
 * d_loss (1 float, may be NULL) receives the loss before the update. */
int pwfs_cnn_train_step(pwfs_cnn_t net, const float* d_x, const float* d_target, const float* d_weights,
                        int32_t B, float lr, float beta1, float beta2, float eps, float* d_loss, void* stream);

/* Release everything (synchronises the device). */
void pwfs_cnn_destroy(pwfs_cnn_t net);

#ifdef __cplusplus
}
#endif

#endif /* PWFS_CNN_H */
