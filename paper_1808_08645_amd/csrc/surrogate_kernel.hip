// Kernels of the learned trace surrogate: every layer is a GEMM on the BF16 matrix cores
// with FP32 accumulation (3-D convolutions through im2col), plus the elementwise pieces of
// training (ReLU backward, bias gradients, MSE loss, Adam).
//
// BF16 values are stored as uint16_t (the upper half of the FP32 bit pattern); FP32 -> BF16
// rounds to nearest even. v_mfma_f32_16x16x16_bf16: lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16] as element j = 0..3 (checked on the device).
#include "surrogate_internal.hpp"

namespace bbw {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));  // inf / nan
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// C[m][n] (=|+=) act(sum_k A(m,k) B(k,n) + bias[n]); A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn].
// A workgroup of 4 waves computes a 64 x 64 block of C, each wave a 32 x 32 quarter as 2 x 2
// MFMA tiles. K advances in tiles of kKT: the workgroup stages the A tile (64 x kKT) and the
// B tile (kKT x 64) in LDS, each with loads whose consecutive threads read consecutive
// addresses along the operand's unit-stride dimension (coalesced whichever way the operand
// is laid out), both stored k-contiguous so that a lane's 4 consecutive k of an MFMA operand
// are one 8-byte LDS read. The next tile's global loads are in flight while the current one
// is multiplied.
// With g.ksplit > 1, workgroup z sums the K range [z kc, (z+1) kc) (kc a multiple of 16) and
// writes its raw partial block to part[z][M][N]; splitk_reduce_kernel adds the slices in order
// and applies the epilogue.
constexpr int kGT = 64, kKT = 32, kKP = kKT + 4;  // tile edge, K tile, padded LDS row (bf16)
constexpr int kLoadsPerThread = kGT * kKT / 256;

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGT][kKP];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGT][kKP];  // [n][k]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t mb = (int64_t)blockIdx.y * kGT, nb = (int64_t)blockIdx.x * kGT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;  // the wave's quarter
  const int r = lane & 15, kq = lane >> 4;
  const int64_t kb = g.ksplit > 1 ? (int64_t)blockIdx.z * g.kc : 0;
  const int64_t ke = g.ksplit > 1 ? (kb + g.kc < g.K ? kb + g.kc : g.K) : g.K;
  // staging order: along k when k is the unit stride, else along the row (m or n)
  const bool a_k = g.sak == 1, b_k = g.sbk == 1;
  auto stage_pos = [](bool along_k, int idx, int& row, int& k) {
    if (along_k) row = idx / kKT, k = idx % kKT;
    else row = idx % kGT, k = idx / kGT;
  };
  uint16_t ra[kLoadsPerThread], rb[kLoadsPerThread];
  auto load_tile = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < kLoadsPerThread; ++i) {
      int row, k;
      stage_pos(a_k, t + 256 * i, row, k);
      const int64_t m = mb + row, ka = k0 + k;
      ra[i] = (m < g.M && ka < ke) ? g.A[m * g.sam + ka * g.sak] : (uint16_t)0;
      stage_pos(b_k, t + 256 * i, row, k);
      const int64_t n = nb + row, kb2 = k0 + k;
      rb[i] = (n < g.N && kb2 < ke) ? g.B[kb2 * g.sbk + n * g.sbn] : (uint16_t)0;
    }
  };
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  if (kb < ke) load_tile(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kKT) {
    __syncthreads();  // the previous tile's operands have been read
#pragma unroll
    for (int i = 0; i < kLoadsPerThread; ++i) {
      int row, k;
      stage_pos(a_k, t + 256 * i, row, k);
      As[row][k] = ra[i];
      stage_pos(b_k, t + 256 * i, row, k);
      Bs[row][k] = rb[i];
    }
    __syncthreads();
    if (k0 + kKT < ke) load_tile(k0 + kKT);
#pragma unroll
    for (int ks = 0; ks < kKT; ks += 16) {
      s4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const s4*>(&As[wm + 16 * i + r][ks + 4 * kq]);
        b[i] = *reinterpret_cast<const s4*>(&Bs[wn + 16 * i + r][ks + 4 * kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  const int64_t m0 = mb + wm, n0 = nb + wn;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + 16 * i + 4 * kq + e, n = n0 + 16 * j + r;
        if (m < g.M && n < g.N && g.ksplit > 1) {
          g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][e];
        } else if (m < g.M && n < g.N) {
          float v = acc[i][j][e];
          float* c = g.C + m * g.ldc + n;
          if (g.accumulate) v += *c;
          if (g.bias) v += g.bias[n];
          if (g.relu) v = v > 0.f ? v : 0.f;
          *c = v;
          if (g.Cbf) g.Cbf[m * g.ldc + n] = to_bf16(v);
        }
      }
}

__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g) {
  const int64_t total = g.M * g.N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / g.N, n = i - m * g.N;
    float v = 0.f;
    for (int z = 0; z < g.ksplit; ++z) v += g.part[(int64_t)z * total + i];
    float* c = g.C + m * g.ldc + n;
    if (g.accumulate) v += *c;
    if (g.bias) v += g.bias[n];
    if (g.relu) v = v > 0.f ? v : 0.f;
    *c = v;
    if (g.Cbf) g.Cbf[m * g.ldc + n] = to_bf16(v);
  }
}

__global__ __launch_bounds__(256) void cast_bf16_kernel(const float* x, uint16_t* y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = to_bf16(x[i]);
}

// im2col of a 3x3x3 convolution, stride 2, padding 1: in [B][D][D][D][C] (BF16),
// out [B * Do^3][Kp] (BF16) with column ((kz*3 + ky)*3 + kx)*C + c, zero beyond 27 C.
__global__ __launch_bounds__(256) void im2col_kernel(const uint16_t* in, uint16_t* out, int B, int D, int C, int Do,
                                                     int Kp) {
  const int64_t total = (int64_t)B * Do * Do * Do * Kp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(i % Kp);
    int64_t row = i / Kp;
    uint16_t v = 0;
    if (col < 27 * C) {
      const int c = col % C, t = col / C;
      const int kx = t % 3, ky = (t / 3) % 3, kz = t / 9;
      const int ox = (int)(row % Do), oy = (int)((row / Do) % Do), oz = (int)((row / ((int64_t)Do * Do)) % Do);
      const int64_t b = row / ((int64_t)Do * Do * Do);
      const int x = 2 * ox - 1 + kx, y = 2 * oy - 1 + ky, z = 2 * oz - 1 + kz;
      if (x >= 0 && x < D && y >= 0 && y < D && z >= 0 && z < D)
        v = in[(((b * D + z) * D + y) * D + x) * C + c];
    }
    out[i] = v;
  }
}

// The adjoint of im2col as a gather: dx[b][z][y][x][c] = sum of dcol entries that read it.
__global__ __launch_bounds__(256) void col2im_kernel(const float* dcol, float* dx, int B, int D, int C, int Do, int Kp) {
  const int64_t total = (int64_t)B * D * D * D * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    int64_t v = i / C;
    const int x = (int)(v % D), y = (int)((v / D) % D), z = (int)((v / ((int64_t)D * D)) % D);
    const int64_t b = v / ((int64_t)D * D * D);
    float s = 0.f;
    for (int kz = 0; kz < 3; ++kz) {
      const int tz = z + 1 - kz;
      if (tz < 0 || (tz & 1) || tz / 2 >= Do) continue;
      for (int ky = 0; ky < 3; ++ky) {
        const int ty = y + 1 - ky;
        if (ty < 0 || (ty & 1) || ty / 2 >= Do) continue;
        for (int kx = 0; kx < 3; ++kx) {
          const int tx = x + 1 - kx;
          if (tx < 0 || (tx & 1) || tx / 2 >= Do) continue;
          const int64_t row = ((b * Do + tz / 2) * Do + ty / 2) * Do + tx / 2;
          s += dcol[row * Kp + ((kz * 3 + ky) * 3 + kx) * C + c];
        }
      }
    }
    dx[i] = s;
  }
}

// dy *= (a > 0): the ReLU derivative, a the layer's output.
__global__ __launch_bounds__(256) void relu_bwd_kernel(float* dy, const float* a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!(a[i] > 0.f)) dy[i] = 0.f;
}

// db[n] = sum_m dy[m][n]: one workgroup per column, rows strided over its threads, then a
// fixed-order tree (deterministic).
__global__ __launch_bounds__(256) void colsum_kernel(const float* dy, float* db, int64_t M, int64_t N) {
  __shared__ float red[256];
  const int64_t n = blockIdx.x;
  float s = 0.f;
  for (int64_t m = threadIdx.x; m < M; m += 256) s += dy[m * N + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[n] = red[0];
}

// Mean squared error over n values: per-block partial sums of (p - t)^2 in FP64 and the
// gradient 2 (p - t) / n.
__global__ __launch_bounds__(256) void mse_kernel(const float* p, const float* t, float* dp, double* partial, int64_t n) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = p[i] - t[i];
    s += (double)d * d;
    dp[i] = 2.f * d / (float)n;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam (Kingma & Ba) with bias correction; refreshes the BF16 copy of the weights.
__global__ __launch_bounds__(256) void adam_kernel(float* w, const float* g, float* m, float* v, uint16_t* wbf, int64_t n,
                                                   float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = to_bf16(wi);
  }
}

unsigned grid1(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

int last() { return (int)hipGetLastError(); }

}  // namespace

int sur_gemm(const GemmArgs& g, void* s) {
  if (g.M <= 0 || g.N <= 0) return 0;
  dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)(g.ksplit > 1 ? g.ksplit : 1));
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, (hipStream_t)s, g);
  if (g.ksplit > 1) {
    int e = last();
    if (e) return e;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid1(g.M * g.N)), dim3(256), 0, (hipStream_t)s, g);
  }
  return last();
}
int sur_cast_bf16(const float* x, uint16_t* y, int64_t n, void* s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(cast_bf16_kernel, dim3(grid1(n)), dim3(256), 0, (hipStream_t)s, x, y, n);
  return last();
}
int sur_im2col(const uint16_t* in, uint16_t* out, int B, int D, int C, int Do, int Kp, void* s) {
  hipLaunchKernelGGL(im2col_kernel, dim3(grid1((int64_t)B * Do * Do * Do * Kp)), dim3(256), 0, (hipStream_t)s, in, out, B,
                     D, C, Do, Kp);
  return last();
}
int sur_col2im(const float* dcol, float* dx, int B, int D, int C, int Do, int Kp, void* s) {
  hipLaunchKernelGGL(col2im_kernel, dim3(grid1((int64_t)B * D * D * D * C)), dim3(256), 0, (hipStream_t)s, dcol, dx, B, D,
                     C, Do, Kp);
  return last();
}
int sur_relu_bwd(float* dy, const float* a, int64_t n, void* s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(grid1(n)), dim3(256), 0, (hipStream_t)s, dy, a, n);
  return last();
}
int sur_colsum(const float* dy, float* db, int64_t M, int64_t N, void* s) {
  if (N <= 0) return 0;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)N), dim3(256), 0, (hipStream_t)s, dy, db, M, N);
  return last();
}
int sur_mse(const float* p, const float* t, float* dp, double* partial, int64_t n, int nblocks, void* s) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, (hipStream_t)s, p, t, dp, partial, n);
  return last();
}
int sur_adam(float* w, const float* g, float* m, float* v, uint16_t* wbf, int64_t n, float lr, float b1, float b2,
             float eps, float c1, float c2, void* s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(adam_kernel, dim3(grid1(n)), dim3(256), 0, (hipStream_t)s, w, g, m, v, wbf, n, lr, b1, b2, eps, c1, c2);
  return last();
}

}  // namespace bbw
