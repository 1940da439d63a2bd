// Y-streaming passes of RandTucker2i: each pass reads the dense tensor once.
//   stream_dual   : TA = Y x_N B_N^T and TB = Y x_{N-1} B_{N-1}^T (one sketch
//                   sweep of Algorithm 3 needs both: every X_n with n < N is
//                   reached from TA, X_N from TB)
//   stream_single : TA = Y x_N Q_N^T (first contraction of the core,
//                   the core projection of Algorithm 3)
// Y is viewed as [A, I_{N-1}, I_N] (A = prod_{p < N-1} I_p).  The first
// pass of a call also produces ||Y||^2 and the non-finite flag.
#pragma once

#include "../../include/rtucker.h"
#include "common.hpp"

namespace rt {

struct StreamCtx {
  const void* y;        // FP32 / FP64 tensor (or BF16 with RT_FLAG_BF16_INPUT)
  uint16_t* ybf16;      // BF16 copy (mixed precision)
  int precision;
  bool bf16_input;
  int64_t A, I1, I2;    // [A, I_{N-1}, I_N]
  int64_t ldy;          // row stride of ybf16 in values: bf16_copy_ld(I2),
                        // or I2 for the caller's BF16 tensor
  void* ws;
  size_t ws_bytes;
  double* norm_partial;  // per-workgroup partial sums of ||Y||^2 (in ws)
  double* norm_out;      // ||Y||^2 (FP64), written by the first pass
  int32_t* nonfinite;    // set to 1 if ||Y||^2 is not finite
};

size_t stream_workspace_bytes(const rt_tucker_desc* d);
StreamCtx make_stream_ctx(const rt_tucker_desc* d, const void* y,
                          uint16_t* ybf16, void* ws, size_t ws_bytes,
                          double* norm_out, int32_t* nonfinite);

// BF16 precision form (stream_bf16.hip)
size_t bf16_stream_workspace_bytes(int64_t A, int64_t I1, int64_t I2);
int bf16_check_shape(int64_t A, int64_t I1, int64_t I2, int K1, int K2,
                     bool bf16_input);
// row stride (values) of the BF16 copy of rows of I2 values: I2 rounded up
// to a multiple of 64
int64_t bf16_copy_ld(int64_t I2);
// stage: profiling stage that brackets the streaming kernel itself.
// TA / TB / C may be null (not computed); C (the slab-local product
// TA x_{N-1} B1^T, [A, K1, K2]) is made only by the column-split pass:
// *c_done tells whether it was.
int bf16_stream_pass(const StreamCtx& c, bool first, const float* B2, int K2,
                     const float* B1, int K1, float* TA, float* TB, float* C, bool* c_done,
                     int stage, hipStream_t s);

// C (nullable): also C = TA x_{N-1} B1^T per slab where the pass can make
// it (the precision form's column-split pass); *c_done says whether it did.
template <typename T>
int stream_dual(const StreamCtx& c, int sweep, const T* B2, int K2,
                const T* B1, int K1, T* TA, T* TB, T* C, bool* c_done, hipStream_t s);
// Core pass: TA = Y x_N B2^T, or (C given and made, *c_done) only
// C = TA x_{N-1} B1^T per slab without writing TA.
template <typename T>
int stream_single(const StreamCtx& c, int sweep, const T* B2, int K2, const T* B1, int K1,
                  T* TA, T* C, bool* c_done, hipStream_t s);

}  // namespace rt
