// Internal declarations of the trace surrogate: its HIP kernels (surrogate_kernel.hip) and the
// host side that runs the network (surrogate.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bbw {

// C[m][n] (=|+=) act(sum_k A(m,k) B(k,n) + bias[n]) with BF16 operands read through strides,
// A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn], FP32 accumulation and output.
struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  float* C;             // [M][ldc]
  uint16_t* Cbf;        // optional BF16 copy of C (same layout), or null
  const float* bias;    // [N] or null
  int64_t M, N, K;
  int64_t sam, sak, sbk, sbn, ldc;
  int32_t accumulate, relu;
  int32_t ksplit;       // > 1: K in slices of kc (multiple of 16), partial blocks in part
  int64_t kc;
  float* part;          // [ksplit][M][N] scratch
};

int sur_gemm(const GemmArgs& g, void* stream);
int sur_cast_bf16(const float* x, uint16_t* y, int64_t n, void* stream);
int sur_im2col(const uint16_t* in, uint16_t* out, int B, int D, int C, int Do, int Kp, void* stream);
int sur_col2im(const float* dcol, float* dx, int B, int D, int C, int Do, int Kp, void* stream);
int sur_relu_bwd(float* dy, const float* a, int64_t n, void* stream);
int sur_colsum(const float* dy, float* db, int64_t M, int64_t N, void* stream);
int sur_mse(const float* p, const float* t, float* dp, double* partial, int64_t n, int nblocks, void* stream);
int sur_adam(float* w, const float* g, float* m, float* v, uint16_t* wbf, int64_t n, float lr, float b1, float b2,
             float eps, float c1, float c2, void* stream);

// Error message shared with the rest of the library (bbwadg_last_error); returns code.
int set_error(int code, const char* fmt, ...);

}  // namespace bbw
