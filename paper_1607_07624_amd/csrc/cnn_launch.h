// cnn_launch.h -- launchers of the CNN kernels (host side of cnn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pwfs {
namespace cnn {

// C(i, j) = alpha (sum_k A(i, k) B(k, j) [+ bias[j]]) [+ beta C(i, j)] [ReLU], bf16
// operands, FP32 accumulation; outputs FP32 (C) and/or bf16 (Cb).
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
};

// part: split-K partial buffer of part_elems floats (NULL disables split-K).
hipError_t gemm(const GemmArgs& g, float* part, size_t part_elems, hipStream_t st);
hipError_t im2col(const uint16_t* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st);
// The same from an FP32 input, each value rounded to bf16 (round to nearest even).
hipError_t im2col_f32(const float* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st);
hipError_t col2im_mask(const float* dcols, int B, int H, int W, int C, const uint16_t* act, float* dz,
                       uint16_t* dzb, hipStream_t st);
hipError_t relu_mask(const float* g, const uint16_t* act, size_t n, float* dz, uint16_t* dzb, hipStream_t st);
hipError_t to_bf16(const float* x, size_t n, uint16_t* y, hipStream_t st);
hipError_t colsum(const float* dz, int rows, int N, float* out, hipStream_t st);
hipError_t mse(const float* pred, const float* target, const float* weights, int n, int n_out, float* dout,
               uint16_t* doutb, float* loss, hipStream_t st);
hipError_t adam(float* w, const float* g, float* m, float* v, uint16_t* wb, size_t n, float lr, float b1, float b2,
                float eps, float c1, float c2, hipStream_t st);
hipError_t fill0(float* p, size_t n, hipStream_t st);
hipError_t prepare(const float* pupils, const float* ref, const int* valid, int nv, int B, int S, float* x,
                   hipStream_t st);

}  // namespace cnn
}  // namespace pwfs
