// cnn_api.cpp -- C ABI of the learned modal reconstructor: parameter and
// workspace management, forward / backward / Adam sequencing.
#include "../../include/pwfs_cnn.h"
#include "../../include/pwfs.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "cnn_launch.h"

using pwfs::cnn::GemmArgs;

namespace pwfs {
int set_last_error(int status, const std::string& msg);   // shared with the sensor ABI (pwfs_last_error)
bool inject_alloc_failure();                              // allocation fault hook (PWFS_FAULT_INJECT)
}

namespace {

enum { PWFS_CNN_ERR_INVALID_ARG = PWFS_ERR_INVALID_ARG, PWFS_CNN_ERR_NO_DEVICE = PWFS_ERR_NO_DEVICE,
       PWFS_CNN_ERR_OOM = PWFS_ERR_OUT_OF_MEMORY, PWFS_CNN_ERR_HIP = PWFS_ERR_HIP };

int fail(int status, const std::string& msg) { return pwfs::set_last_error(status, msg); }
int hip_fail(hipError_t e, const char* what) {
  return fail(PWFS_CNN_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) return 0;
  if (pwfs::inject_alloc_failure()) return fail(PWFS_CNN_ERR_OOM, std::string("injected OOM: ") + what);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(PWFS_CNN_ERR_OOM, std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
  }
  return 0;
}

}  // namespace

struct pwfs_cnn_s {
  pwfs_cnn_config_t cfg{};
  int device = 0;
  int S = 0, S1 = 0, S2 = 0, S3 = 0, c1 = 0, c2 = 0, c3 = 0, hidden = 0, nout = 0, flat = 0, bm = 0;
  size_t off[10] = {};   // w1 b1 w2 b2 w3 b3 fw1 fb1 fw2 fb2
  size_t n_params = 0;
  pwfs::cnn::ConvPerm cperm{};   // convolution blocks of the bf16 product copy
  long step = 0;
  // parameters
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t* wb = nullptr;
  // activations as bf16 pairs (lo plane after the hi plane; cols1, the
  // bf16-rounded input's im2col, is one plane) and FP32 work buffers
  uint16_t *cols1 = nullptr, *a1 = nullptr, *cols2 = nullptr, *a2 = nullptr, *cols3 = nullptr,
           *a3 = nullptr, *h = nullptr, *doutb = nullptr, *dzf = nullptr;
  // upstream gradients of the three convolutions' outputs (bf16 pairs), one
  // buffer per layer so that a layer's weight gradient can still read its
  // own while the data gradients move on
  uint16_t *dz3 = nullptr, *dz2 = nullptr, *dz1 = nullptr;
  float *out = nullptr, *gtmp = nullptr, *part = nullptr, *part2 = nullptr, *loss = nullptr, *mse_part = nullptr;
  size_t part_elems = 0;
  // backward: the weight gradients run on `side` (default priority) beside
  // the chain of data gradients on the caller's stream; ev fork and join
  hipStream_t side = nullptr;
  hipEvent_t ev[6] = {};
};

namespace {

void free_net(pwfs_cnn_s* n) {
  if (!n) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(n->device);
  if (n->side) (void)hipStreamSynchronize(n->side);
  for (hipEvent_t e : n->ev)
    if (e) (void)hipEventDestroy(e);
  if (n->side) (void)hipStreamDestroy(n->side);
  void* ptrs[] = {n->w, n->m, n->v, n->g, n->wb, n->cols1, n->a1, n->cols2, n->a2, n->cols3, n->a3,
                  n->h, n->doutb, n->dzf, n->dz3, n->dz2, n->dz1, n->out, n->gtmp, n->part, n->part2,
                  n->loss, n->mse_part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete n;
}

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != d) (void)hipSetDevice(d);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define CK(expr)                                  \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

// Y = X W^T + bias (ReLU), X [M][K] bf16 (a pair when x_split: lo plane M K
// elements on), W [N][K] bf16; Y to C (FP32) and/or Cb (a bf16 pair, lo
// plane M N elements on).
GemmArgs fwd_args(const uint16_t* X, bool x_split, const uint16_t* W, const float* bias, int M, int N, int K,
                  bool relu, float* C, uint16_t* Cb) {
  GemmArgs a{};
  a.A = X; a.sam = K; a.sak = 1; a.a_lo = x_split ? (long)M * K : 0;
  a.B = W; a.sbk = 1; a.sbn = K;
  a.C = C; a.ldc = N; a.Cb = Cb; a.ldcb = N; a.cb_lo = Cb ? (long)M * N : 0;
  a.bias = bias; a.M = M; a.N = N; a.K = K; a.alpha = 1.f; a.beta = 0.f; a.relu = relu ? 1 : 0;
  return a;
}
// dW [N][K] = dY^T X and db [N] = column sums of dY; dY [R][N] a bf16 pair
// (lo plane R N elements on), X [R][K] bf16 (a pair when x_split).
GemmArgs wgrad_args(const uint16_t* dY, const uint16_t* X, bool x_split, int R, int N, int K, float* dW, float* db,
                    int cperm = 0) {
  GemmArgs a{};
  a.cperm = cperm;   // convolutions: patch columns (tap, c) go to weight columns (c, tap)
  a.A = dY; a.sam = 1; a.sak = N; a.a_lo = (long)R * N;
  a.B = X; a.sbk = K; a.sbn = 1; a.b_lo = x_split ? (long)R * K : 0;
  a.C = dW; a.ldc = K; a.bias_grad = db;
  a.M = N; a.N = K; a.K = R; a.alpha = 1.f;
  return a;
}
// dX [R][K] = dY W, dY [R][N] a bf16 pair, W [N][K] bf16.
GemmArgs dgrad_args(const uint16_t* dY, const uint16_t* W, int R, int N, int K, float* dX) {
  GemmArgs a{};
  a.A = dY; a.sam = N; a.sak = 1; a.a_lo = (long)R * N;
  a.B = W; a.sbk = K; a.sbn = 1;
  a.C = dX; a.ldc = K;
  a.M = R; a.N = K; a.K = N; a.alpha = 1.f;
  return a;
}

// dX = (dY W) masked by act > 0 (act [R][K], the hi plane of the layer's input
// activation), as a bf16 pair [R][K] (lo plane R K elements on); dX must not
// alias dY.
GemmArgs dgrad_masked_args(const uint16_t* dY, const uint16_t* W, int R, int N, int K, const uint16_t* act,
                           uint16_t* dX) {
  GemmArgs a = dgrad_args(dY, W, R, N, K, nullptr);
  a.ldc = 0;
  a.Cb = dX; a.ldcb = K; a.cb_lo = (long)R * K;
  a.mask = act; a.ldm = K;
  return a;
}

// Convolutions of the tiled products read their patches straight from the
// activation (implicit im2col) when its channel count is a multiple of 8 and
// the product is tall enough for the tiled kernel; otherwise (few frames: the
// matrix-vector kernel; other channel counts) the patches are gathered first.
bool implicit_patches(int C, int rows) { return C % 8 == 0 && rows > 512; }

// Forward product of a convolution on implicit patches of act [B][H][W][C]
// (bf16 pair, lo plane B H W C elements on).
GemmArgs fwd_conv_args(const uint16_t* act, int H, int W, int C, const uint16_t* Wt, const float* bias, int M, int N,
                       uint16_t* Cb, int B) {
  GemmArgs a = fwd_args(act, true, Wt, bias, M, N, 9 * C, true, nullptr, Cb);
  a.a_lo = (long)B * H * W * C;
  a.sam = 0;
  a.conv_op = 1; a.conv_H = H; a.conv_W = W; a.conv_C = C;
  return a;
}

// Weight gradient of a convolution with its input patches implicit in act
// [B][H][W][C] (bf16 pair); dY [R][N] pair as in wgrad_args.
GemmArgs wgrad_conv_args(const uint16_t* dY, const uint16_t* act, int H, int W, int C, int R, int N, float* dW,
                         float* db, int B) {
  GemmArgs a = wgrad_args(dY, act, true, R, N, 9 * C, dW, db, C);
  a.b_lo = (long)B * H * W * C;
  a.sbk = 0;
  a.conv_op = 2; a.conv_H = H; a.conv_W = W; a.conv_C = C;
  return a;
}

// Forward pass; the last layer writes out_alpha * net(x) + out_beta * out into
// `out` (NULL: the internal output buffer, alpha 1, beta 0).
// The two fully connected layers, from the third convolution's output pair.
int run_dense(pwfs_cnn_s* n, int B, hipStream_t st, float* out, float out_alpha, float out_beta) {
  const float* W = n->w;
  const uint16_t* Wb = n->wb;
  CK(pwfs::cnn::gemm(fwd_args(n->a3, true, Wb + n->off[6], W + n->off[7], B, n->hidden, n->flat, true, nullptr, n->h),
                     n->part, n->part_elems, st));
  GemmArgs last = fwd_args(n->h, true, Wb + n->off[8], W + n->off[9], B, n->nout, n->hidden, false,
                           out ? out : n->out, nullptr);
  if (out) {
    last.alpha = out_alpha;
    last.beta = out_beta;
  }
  CK(pwfs::cnn::gemm(last, n->part, n->part_elems, st));
  return 0;
}

// Forward pass: the three convolutions as one block per frame
// (pwfs::cnn::conv_stack) when the shapes allow it, else a patch gather and
// a tiled product per layer; a training step keeps every activation its
// backward pass reads, a forward-only call (inference) only the third
// convolution's output.
int run_forward(pwfs_cnn_s* n, const float* x, int B, hipStream_t st, float* out = nullptr,
                float out_alpha = 1.f, float out_beta = 0.f, bool inference = false) {
  const float* W = n->w;
  const uint16_t* Wb = n->wb;
  const int R1 = B * n->S1 * n->S1, R2 = B * n->S2 * n->S2, R3 = B * n->S3 * n->S3;
  // the convolutions as one block per frame; a training step also keeps the
  // first layer's patches and the first two activation pairs (its backward
  // pass reads the second and third layers' patches from them)
  const bool keep = !inference;
  const hipError_t cs = pwfs::cnn::conv_stack(
      x, B, n->S, Wb + n->off[0], W + n->off[1], n->c1, Wb + n->off[2], W + n->off[3], n->c2, Wb + n->off[4],
      W + n->off[5], n->c3, n->a3, (long)R3 * n->c3, st, keep ? n->cols1 : nullptr, keep ? n->a1 : nullptr,
      (long)R1 * n->c1, keep ? n->a2 : nullptr, (long)R2 * n->c2);
  if (cs != hipSuccess && cs != hipErrorNotSupported) return hip_fail(cs, "cnn convolution stack");
  if (cs == hipSuccess) return run_dense(n, B, st, out, out_alpha, out_beta);
  CK(pwfs::cnn::im2col_f32(x, B, n->S, n->S, 4, n->cols1, st));   // input rounded to bf16 on the way
  CK(pwfs::cnn::gemm(fwd_args(n->cols1, false, Wb + n->off[0], W + n->off[1], R1, n->c1, 36, true, nullptr, n->a1),
                     n->part, n->part_elems, st));
  if (implicit_patches(n->c1, R2)) {
    CK(pwfs::cnn::gemm(fwd_conv_args(n->a1, n->S1, n->S1, n->c1, Wb + n->off[2], W + n->off[3], R2, n->c2, n->a2, B),
                       n->part, n->part_elems, st));
  } else {
    CK(pwfs::cnn::im2col(n->a1, B, n->S1, n->S1, n->c1, n->cols2, st));
    CK(pwfs::cnn::gemm(fwd_args(n->cols2, true, Wb + n->off[2], W + n->off[3], R2, n->c2, n->c1 * 9, true, nullptr,
                                n->a2), n->part, n->part_elems, st));
  }
  if (implicit_patches(n->c2, R3)) {
    CK(pwfs::cnn::gemm(fwd_conv_args(n->a2, n->S2, n->S2, n->c2, Wb + n->off[4], W + n->off[5], R3, n->c3, n->a3, B),
                       n->part, n->part_elems, st));
  } else {
    CK(pwfs::cnn::im2col(n->a2, B, n->S2, n->S2, n->c2, n->cols3, st));
    CK(pwfs::cnn::gemm(fwd_args(n->cols3, true, Wb + n->off[4], W + n->off[5], R3, n->c3, n->c2 * 9, true, nullptr,
                                n->a3), n->part, n->part_elems, st));
  }
  return run_dense(n, B, st, out, out_alpha, out_beta);
}

// Adam hyper-parameters and bias corrections of one training step.
struct AdamStep {
  float lr, b1, b2, eps, c1, c2;
};

// Backward pass.  The data gradients form a chain on the caller's stream
// (each layer's needs the one above); a layer's weight gradient needs only
// that layer's upstream gradient and its forward input, and nothing reads it
// before the optimiser, so the weight gradients run on the side stream, each
// after an event on the chain, and the caller's stream waits for the side
// stream at the end.  Each product alone leaves most of the GPU idle (a few
// hundred blocks of a few k steps), so the two streams overlap.  The first
// layer's weight gradient stays on the chain, which has no other work left
// by then; the loss sum (read by nothing in the step) goes to the side stream.
// With opt (a training step), the Adam update of every parameter but the
// first layer's runs on the side stream after its last weight gradient and
// after the chain's last read of those weights (the second convolution's
// data gradient), beside the chain's first-layer weight gradient; the chain
// then updates the first layer.
int run_backward(pwfs_cnn_s* n, const float* target, const float* weights, int B, float* loss, hipStream_t st,
                 const AdamStep* opt = nullptr) {
  const uint16_t* Wb = n->wb;
  float* G = n->g;
  const size_t P = (size_t)n->part_elems;
  hipStream_t sd = n->side;
  auto fork = [&](int e) -> hipError_t {   // side stream continues after everything queued on st so far
    hipError_t r = hipEventRecord(n->ev[e], st);
    return r != hipSuccess ? r : hipStreamWaitEvent(sd, n->ev[e], 0);
  };
  const int R3 = B * n->S3 * n->S3, R2 = B * n->S2 * n->S2, R1 = B * n->S1 * n->S1;
  CK(pwfs::cnn::mse(n->out, target, weights, B * n->nout, n->nout, n->doutb, n->mse_part, st));
  // fc2: weight gradient (side, after the loss sum); data gradient with the ReLU mask of h (chain)
  CK(fork(0));
  CK(pwfs::cnn::mse_sum(n->mse_part, B * n->nout, loss, sd));
  CK(pwfs::cnn::gemm(wgrad_args(n->doutb, n->h, true, B, n->nout, n->hidden, G + n->off[8], G + n->off[9]),
                     n->part2, P, sd));
  CK(pwfs::cnn::gemm(dgrad_masked_args(n->doutb, Wb + n->off[8], B, n->nout, n->hidden, n->h, n->dzf), n->part, P,
                     st));
  // fc1
  CK(fork(1));
  CK(pwfs::cnn::gemm(wgrad_args(n->dzf, n->a3, true, B, n->hidden, n->flat, G + n->off[6], G + n->off[7]),
                     n->part2, P, sd));
  CK(pwfs::cnn::gemm(dgrad_masked_args(n->dzf, Wb + n->off[6], B, n->hidden, n->flat, n->a3, n->dz3), n->part, P,
                     st));
  // conv3
  CK(fork(2));
  if (n->c2 % 8 == 0)
    CK(pwfs::cnn::gemm(wgrad_conv_args(n->dz3, n->a2, n->S2, n->S2, n->c2, R3, n->c3, G + n->off[4], G + n->off[5], B),
                       n->part2, P, sd));
  else
    CK(pwfs::cnn::gemm(wgrad_args(n->dz3, n->cols3, true, R3, n->c3, n->c2 * 9, G + n->off[4], G + n->off[5], n->c2),
                       n->part2, P, sd));
  CK(pwfs::cnn::gemm(dgrad_args(n->dz3, Wb + n->off[4], R3, n->c3, n->c2 * 9, n->gtmp), n->part, P, st));
  CK(pwfs::cnn::col2im_mask(n->gtmp, B, n->S2, n->S2, n->c2, n->a2, n->dz2, st));
  // conv2
  CK(fork(3));
  if (n->c1 % 8 == 0)
    CK(pwfs::cnn::gemm(wgrad_conv_args(n->dz2, n->a1, n->S1, n->S1, n->c1, R2, n->c2, G + n->off[2], G + n->off[3], B),
                       n->part2, P, sd));
  else
    CK(pwfs::cnn::gemm(wgrad_args(n->dz2, n->cols2, true, R2, n->c2, n->c1 * 9, G + n->off[2], G + n->off[3], n->c1),
                       n->part2, P, sd));
  CK(pwfs::cnn::gemm(dgrad_args(n->dz2, Wb + n->off[2], R2, n->c2, n->c1 * 9, n->gtmp), n->part, P, st));
  if (opt) {
    CK(hipEventRecord(n->ev[5], st));   // the chain's last read of the weights past the first layer
    CK(hipStreamWaitEvent(sd, n->ev[5], 0));
    CK(pwfs::cnn::adam(n->w, n->g, n->m, n->v, n->wb, n->cperm, n->off[2], n->n_params, opt->lr, opt->b1, opt->b2,
                       opt->eps, opt->c1, opt->c2, sd));
  }
  CK(pwfs::cnn::col2im_mask(n->gtmp, B, n->S1, n->S1, n->c1, n->a1, n->dz1, st));
  // conv1: weight gradient only, on the chain
  CK(pwfs::cnn::gemm(wgrad_args(n->dz1, n->cols1, false, R1, n->c1, 36, G + n->off[0], G + n->off[1], 4),
                     n->part, P, st));
  if (opt)
    CK(pwfs::cnn::adam(n->w, n->g, n->m, n->v, n->wb, n->cperm, 0, n->off[2], opt->lr, opt->b1, opt->b2, opt->eps,
                       opt->c1, opt->c2, st));
  // join
  CK(hipEventRecord(n->ev[4], sd));
  CK(hipStreamWaitEvent(st, n->ev[4], 0));
  return 0;
}

int check_batch(pwfs_cnn_s* n, int B) {
  if (!n) return fail(PWFS_CNN_ERR_INVALID_ARG, "network is NULL");
  if (B < 0 || B > n->bm) return fail(PWFS_CNN_ERR_INVALID_ARG, "B must be in [0, batch_max]");
  return 0;
}

}  // namespace

extern "C" {

int pwfs_cnn_create(const pwfs_cnn_config_t* c, pwfs_cnn_t* out) {
  if (!out) return fail(PWFS_CNN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!c) return fail(PWFS_CNN_ERR_INVALID_ARG, "cfg is NULL");
  if (c->reserved != 0 || c->n_sub < 4 || c->n_sub > 256 || c->c1 < 1 || c->c1 > 256 || c->c2 < 1 ||
      c->c2 > 256 || c->c3 < 1 || c->c3 > 256 || c->hidden < 1 || c->hidden > 16384 || c->n_out < 1 ||
      c->n_out > 16384 || c->batch_max < 1 || c->batch_max > 65535)
    return fail(PWFS_CNN_ERR_INVALID_ARG, "configuration out of range");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(PWFS_CNN_ERR_NO_DEVICE, "no HIP device visible");
  }
  auto* n = new pwfs_cnn_s();
  n->cfg = *c;
  (void)hipGetDevice(&n->device);
  n->S = c->n_sub;
  n->S1 = (n->S + 1) / 2;
  n->S2 = (n->S1 + 1) / 2;
  n->S3 = (n->S2 + 1) / 2;
  n->c1 = c->c1; n->c2 = c->c2; n->c3 = c->c3;
  n->hidden = c->hidden; n->nout = c->n_out; n->bm = c->batch_max;
  n->flat = n->S3 * n->S3 * n->c3;
  const size_t sizes[10] = {(size_t)n->c1 * 4 * 9, (size_t)n->c1, (size_t)n->c2 * n->c1 * 9, (size_t)n->c2,
                            (size_t)n->c3 * n->c2 * 9, (size_t)n->c3, (size_t)n->hidden * n->flat,
                            (size_t)n->hidden, (size_t)n->nout * n->hidden, (size_t)n->nout};
  size_t o = 0;
  for (int i = 0; i < 10; ++i) {
    n->off[i] = o;
    o += sizes[i];   // packed, C order
  }
  n->n_params = o;
  n->cperm = pwfs::cnn::ConvPerm{{n->off[0], n->off[2], n->off[4]}, {4, n->c1, n->c2}, {n->c1, n->c2, n->c3}};
  const size_t B = (size_t)n->bm;
  const size_t R1 = B * n->S1 * n->S1, R2 = B * n->S2 * n->S2, R3 = B * n->S3 * n->S3;
  const size_t gtmp = std::max({B * n->hidden, B * n->flat, R3 * n->c2 * 9, R2 * n->c1 * 9});
  n->part_elems = std::max<size_t>({(size_t)4 << 20, (size_t)64 * n->c1 * 36, (size_t)64 * n->c2 * n->c1 * 9,
                                    (size_t)64 * n->c3 * n->c2 * 9});
  struct A { void** p; size_t bytes; const char* what; } al[] = {
      {(void**)&n->w, n->n_params * 4, "params"}, {(void**)&n->m, n->n_params * 4, "adam m"},
      {(void**)&n->v, n->n_params * 4, "adam v"}, {(void**)&n->g, n->n_params * 4, "grads"},
      {(void**)&n->wb, n->n_params * 2, "bf16 params"},
      {(void**)&n->cols1, R1 * 36 * 2, "cols1"},
      {(void**)&n->a1, R1 * n->c1 * 2 * 2, "a1 pair"}, {(void**)&n->cols2, R2 * n->c1 * 9 * 2 * 2, "cols2 pair"},
      {(void**)&n->a2, R2 * n->c2 * 2 * 2, "a2 pair"}, {(void**)&n->cols3, R3 * n->c2 * 9 * 2 * 2, "cols3 pair"},
      {(void**)&n->a3, R3 * n->c3 * 2 * 2, "a3 pair"}, {(void**)&n->h, B * n->hidden * 2 * 2, "hidden pair"},
      {(void**)&n->doutb, B * n->nout * 2 * 2, "dout pair"},
      {(void**)&n->dzf, B * n->hidden * 2 * 2, "hidden-layer dz pair"},
      {(void**)&n->dz3, R3 * n->c3 * 2 * 2, "conv3 dz pair"}, {(void**)&n->dz2, R2 * n->c2 * 2 * 2, "conv2 dz pair"},
      {(void**)&n->dz1, R1 * n->c1 * 2 * 2, "conv1 dz pair"},
      {(void**)&n->out, B * n->nout * 4, "out"},
      {(void**)&n->gtmp, gtmp * 4, "data gradients"},
      {(void**)&n->part, n->part_elems * 4, "split-K partials"},
      {(void**)&n->part2, n->part_elems * 4, "split-K partials (side stream)"}, {(void**)&n->loss, 4, "loss"},
      {(void**)&n->mse_part, pwfs::cnn::mse_partials((int)(B * n->nout)) * 4, "loss partials"},
  };
  for (auto& a : al) {
    int s = dev_alloc(a.p, a.bytes, a.what);
    if (s) {
      free_net(n);
      return s;
    }
  }
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&n->side, hipStreamNonBlocking)) != hipSuccess) {
    n->side = nullptr;
    free_net(n);
    return hip_fail(e, "pwfs_cnn_create (side stream)");
  }
  for (hipEvent_t& ev : n->ev) {
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
      ev = nullptr;
      free_net(n);
      return hip_fail(e, "pwfs_cnn_create (events)");
    }
  }
  if ((e = hipMemset(n->w, 0, n->n_params * 4)) != hipSuccess || (e = hipMemset(n->m, 0, n->n_params * 4)) != hipSuccess ||
      (e = hipMemset(n->v, 0, n->n_params * 4)) != hipSuccess || (e = hipMemset(n->wb, 0, n->n_params * 2)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    free_net(n);
    return hip_fail(e, "pwfs_cnn_create");
  }
  *out = n;
  return 0;
}

int pwfs_cnn_num_params(pwfs_cnn_t n, int64_t* np) {
  if (!n || !np) return fail(PWFS_CNN_ERR_INVALID_ARG, "network or output is NULL");
  *np = (int64_t)n->n_params;
  return 0;
}

int pwfs_cnn_set_params(pwfs_cnn_t n, const float* d, void* stream) {
  if (!n || !d) return fail(PWFS_CNN_ERR_INVALID_ARG, "network or params is NULL");
  DevGuard g(n->device);
  hipStream_t st = (hipStream_t)stream;
  CK(hipMemcpyAsync(n->w, d, n->n_params * 4, hipMemcpyDeviceToDevice, st));
  CK(pwfs::cnn::weights_bf16(n->w, n->n_params, n->cperm, n->wb, st));
  CK(pwfs::cnn::fill0(n->m, n->n_params, st));
  CK(pwfs::cnn::fill0(n->v, n->n_params, st));
  n->step = 0;
  return 0;
}

int pwfs_cnn_get_params(pwfs_cnn_t n, float* d, void* stream) {
  if (!n || !d) return fail(PWFS_CNN_ERR_INVALID_ARG, "network or params is NULL");
  DevGuard g(n->device);
  CK(hipMemcpyAsync(d, n->w, n->n_params * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return 0;
}

int pwfs_cnn_get_optimizer(pwfs_cnn_t n, float* d_m, float* d_v, int64_t* step, void* stream) {
  if (!n || !d_m || !d_v || !step) return fail(PWFS_CNN_ERR_INVALID_ARG, "network or output is NULL");
  DevGuard g(n->device);
  hipStream_t st = (hipStream_t)stream;
  CK(hipMemcpyAsync(d_m, n->m, n->n_params * 4, hipMemcpyDeviceToDevice, st));
  CK(hipMemcpyAsync(d_v, n->v, n->n_params * 4, hipMemcpyDeviceToDevice, st));
  *step = (int64_t)n->step;
  return 0;
}

int pwfs_cnn_set_optimizer(pwfs_cnn_t n, const float* d_m, const float* d_v, int64_t step, void* stream) {
  if (!n || !d_m || !d_v) return fail(PWFS_CNN_ERR_INVALID_ARG, "network or state is NULL");
  if (step < 0) return fail(PWFS_CNN_ERR_INVALID_ARG, "step must be >= 0");
  DevGuard g(n->device);
  hipStream_t st = (hipStream_t)stream;
  CK(hipMemcpyAsync(n->m, d_m, n->n_params * 4, hipMemcpyDeviceToDevice, st));
  CK(hipMemcpyAsync(n->v, d_v, n->n_params * 4, hipMemcpyDeviceToDevice, st));
  n->step = (long)step;
  return 0;
}

int pwfs_cnn_prepare(const float* d_pupils, const float* d_ref, const int32_t* d_valid, int32_t nv, int32_t B,
                     int32_t S, float* d_x, void* stream) {
  if (B < 0 || nv <= 0 || S <= 0 || nv > S * S) return fail(PWFS_CNN_ERR_INVALID_ARG, "bad sizes");
  if (B == 0) return 0;
  if (!d_pupils || !d_ref || !d_valid || !d_x) return fail(PWFS_CNN_ERR_INVALID_ARG, "NULL pointer");
  CK(pwfs::cnn::prepare(d_pupils, d_ref, d_valid, nv, B, S, d_x, (hipStream_t)stream));
  return 0;
}

int pwfs_cnn_forward(pwfs_cnn_t n, const float* d_x, int32_t B, float* d_out, void* stream) {
  int s = check_batch(n, B);
  if (s) return s;
  if (B == 0) return 0;
  if (!d_x || !d_out) return fail(PWFS_CNN_ERR_INVALID_ARG, "NULL pointer");
  DevGuard g(n->device);
  hipStream_t st = (hipStream_t)stream;
  return run_forward(n, d_x, B, st, d_out, 1.f, 0.f, true);
}

int pwfs_cnn_forward_acc(pwfs_cnn_t n, const float* d_x, int32_t B, float alpha, float beta, float* d_out,
                         void* stream) {
  int s = check_batch(n, B);
  if (s) return s;
  if (B == 0) return 0;
  if (!d_x || !d_out) return fail(PWFS_CNN_ERR_INVALID_ARG, "NULL pointer");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(PWFS_CNN_ERR_INVALID_ARG, "alpha/beta not finite");
  DevGuard g(n->device);
  return run_forward(n, d_x, B, (hipStream_t)stream, d_out, alpha, beta, true);
}

int pwfs_cnn_gradients(pwfs_cnn_t n, const float* d_x, const float* d_target, const float* d_weights, int32_t B,
                       float* d_grads, float* d_loss, void* stream) {
  int s = check_batch(n, B);
  if (s) return s;
  if (B == 0) return 0;
  if (!d_x || !d_target) return fail(PWFS_CNN_ERR_INVALID_ARG, "NULL pointer");
  DevGuard g(n->device);
  hipStream_t st = (hipStream_t)stream;
  if ((s = run_forward(n, d_x, B, st))) return s;
  if ((s = run_backward(n, d_target, d_weights, B, d_loss ? d_loss : n->loss, st))) return s;
  if (d_grads) CK(hipMemcpyAsync(d_grads, n->g, n->n_params * 4, hipMemcpyDeviceToDevice, st));
  return 0;
}

int pwfs_cnn_train_step(pwfs_cnn_t n, const float* d_x, const float* d_target, const float* d_weights, int32_t B,
                        float lr, float beta1, float beta2, float eps, float* d_loss, void* stream) {
  int s = check_batch(n, B);
  if (s) return s;
  if (B == 0) return 0;
  if (!d_x || !d_target) return fail(PWFS_CNN_ERR_INVALID_ARG, "NULL pointer");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(PWFS_CNN_ERR_INVALID_ARG, "optimizer hyper-parameters out of range");
  DevGuard g(n->device);
  hipStream_t st = (hipStream_t)stream;
  if ((s = run_forward(n, d_x, B, st))) return s;
  const long step = n->step + 1;
  const AdamStep opt{lr, beta1, beta2, eps, (float)(1.0 - std::pow((double)beta1, (double)step)),
                     (float)(1.0 - std::pow((double)beta2, (double)step))};
  if ((s = run_backward(n, d_target, d_weights, B, d_loss ? d_loss : n->loss, st, &opt))) return s;
  n->step = step;
  return 0;
}

void pwfs_cnn_destroy(pwfs_cnn_t n) {
  if (!n) return;
  {
    DevGuard g(n->device);
    (void)hipDeviceSynchronize();
  }
  free_net(n);
}

}  // extern "C"
