// cnn_launch.h -- launchers of the CNN kernels (host side of cnn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pwfs {
namespace cnn {

// C(i, j) = alpha (sum_k A(i, k) B(k, j) [+ bias[j]]) [+ beta C(i, j)] [ReLU], bf16
// operands, FP32 accumulation; outputs FP32 (C) and/or bf16 (Cb).
// A(i, k) = A[i sam + k sak], B(k, j) = B[k sbk + j sbn].
// Split operands: with a_lo != 0 the operand A is the bf16 pair hi + lo, the
// lo plane at A + a_lo (same strides); likewise b_lo for B.  The product is
// A_hi B_hi + A_lo B_hi + A_hi B_lo (the lo x lo term, below 2^-16 of the
// product, is left out).  With cb_lo != 0 the bf16 output is written as a
// pair too: Cb = bf16(x), Cb[. + cb_lo] = bf16(x - Cb).
// bias_grad: an extra output column j = N with B(k, N) = 1 (hi plane; 0 in
// the lo plane), i.e. bias_grad[i] = sum_k A(i, k), written raw.
struct GemmArgs {
  const uint16_t* A;
  long sam, sak;
  const uint16_t* B;
  long sbk, sbn;
  float* C;
  long ldc;
  uint16_t* Cb;
  long ldcb;
  const float* bias;
  int M, N, K;
  float alpha;
  float beta;
  int relu;
  long a_lo, b_lo, cb_lo;
  float* bias_grad;
  int cperm;          // > 0: output column j (patch order tap, c) is stored at (j mod cperm) 9 + j / cperm
  const uint16_t* mask;   // ReLU mask: output (i, j) is zeroed unless mask[i ldm + j] (bf16) > 0; NULL: none
  long ldm;
  // Implicit patches of a 3x3 stride-2 pad-1 convolution (C a multiple of 8):
  // conv_op 1: A is the NHWC activation [B][H][W][C] (its lo plane a_lo on)
  // read as patches A(i = output pixel, k = (ky, kx, c)); conv_op 2: B is that
  // activation read as B(j = (ky, kx, c), k = output pixel).  0: none.
  int conv_op, conv_H, conv_W, conv_C;
};

// The three convolution weight blocks of the flat parameter vector (offset,
// input and output channels): their bf16 product copy is stored
// [Cout][3][3][Cin] (patch order of im2col), the FP32 weights [Cout][Cin][3][3].
struct ConvPerm {
  size_t off[3];
  int cin[3], cout[3];
};

// part: split-K partial buffer of part_elems floats (NULL disables split-K).
hipError_t gemm(const GemmArgs& g, float* part, size_t part_elems, hipStream_t st);
// Patches in (ky, kx, c) order.  Activations are bf16 pairs: the lo plane of
// act (cols) lies n elements after its hi plane, n the plane's element count.
hipError_t im2col(const uint16_t* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st);
// The same from an FP32 input, each value rounded to bf16 (round to nearest even).
hipError_t im2col_f32(const float* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st);
// Data gradients masked by the forward output's ReLU, written as bf16 pairs
// (lo plane after the hi plane).
hipError_t col2im_mask(const float* dcols, int B, int H, int W, int C, const uint16_t* act, uint16_t* dzb,
                       hipStream_t st);
// bf16 product copy of the FP32 parameters (convolution weights permuted as in ConvPerm).
hipError_t weights_bf16(const float* x, size_t n, const ConvPerm& cp, uint16_t* y, hipStream_t st);
// part: at least mse_partials(n) floats of scratch.  mse writes the gradient
// pair and the per-block partial sums; mse_sum (on any stream ordered after
// mse) adds the partials in block order into the loss.
size_t mse_partials(int n);
hipError_t mse(const float* pred, const float* target, const float* weights, int n, int n_out, uint16_t* doutb,
               float* part, hipStream_t st);
hipError_t mse_sum(const float* part, int n, float* loss, hipStream_t st);
// Adam on the parameters [i0, n) of the flat vector (indices absolute).
hipError_t adam(float* w, const float* g, float* m, float* v, uint16_t* wb, const ConvPerm& cp, size_t i0, size_t n,
                float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t fill0(float* p, size_t n, hipStream_t st);
// The three convolutions of a forward-only call, one block per frame:
// x [B][S][S][4] FP32 -> a3 pair (lo plane a3_lo on), bf16 weights in patch
// order.  hipErrorNotSupported (nothing launched) when the shapes are
// outside the kernel's limits: 32 first-layer and 32 or 64 second-layer
// channels, a multiple of 32 in the third, the staged activations within
// 64 KiB of LDS, a 16-byte aligned input and weights of the second and
// third layers.
bool conv_stack_fits(int S, int c1, int c2, int c3);
// cols1 [B M1][36], a1 and a2 (pairs, lo planes a1_lo / a2_lo on): the first
// layer's patches and the first two activation pairs for a training step's
// backward pass; NULL: not written.
hipError_t conv_stack(const float* x, int B, int S, const uint16_t* w1, const float* b1, int c1, const uint16_t* w2,
                      const float* b2, int c2, const uint16_t* w3, const float* b3, int c3, uint16_t* a3, long a3_lo,
                      hipStream_t st, uint16_t* cols1 = nullptr, uint16_t* a1 = nullptr, long a1_lo = 0,
                      uint16_t* a2 = nullptr, long a2_lo = 0);
hipError_t prepare(const float* pupils, const float* ref, const int* valid, int nv, int B, int S, float* x,
                   hipStream_t st);

}  // namespace cnn
}  // namespace pwfs
