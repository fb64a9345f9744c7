// Dense quadrature WADG update (paper Section 3.3, eq. pwadg) on the matrix cores (FP64, or
// FP32 with FP32 accumulation):
//     out = P_q diag(c^2(x_q)) V_q r
// per element, with V_q the Bernstein basis at the Nq points of a collapsed Gauss-Jacobi
// rule and P_q = M^{-1} V_q^T W the quadrature L^2 projection. It is the comparison
// baseline of the fast Bernstein update: O(Nq Np) = O(N^6) work per element instead of
// O(N^4), and Nq values of c^2 stored per element instead of Mp coefficients.
//
// Both products are dense contractions shared by all elements, so a wavefront takes a
// tile of 16 elements and runs them on v_mfma_f64_16x16x4f64 (v_mfma_f32_16x16x4f32):
//   U (16 points x 16 elements) = V_q[chunk] (16 x Np) . R (Np x 16)       Np/4 MFMAs
//   U *= c^2 at those points (per element)
//   Out (Np x 16) += P_q[:, chunk] (Np x 16) . U (16 x 16)                  Np/4 MFMAs
// over the point chunks. The tables are stored in the MFMA operand order (one coalesced
// 512-byte load per operand, L2-resident); R and U pass through LDS to change from the
// accumulator layout to the B-operand layout. Lane l holds A[l%16][l/16] and B[l/16][l%16];
// it holds D[4i + l/16][l%16] (FP64, checked on the device) or D[4(l/16) + i][l%16] (FP32, the
// layout of the FP32-output 16x16 instructions, checked on the device for the BF16 one) as
// element i = 0..3 of its result.
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename real> struct Acc4;
template <> struct Acc4<double> { typedef d4 type; };
template <> struct Acc4<float> { typedef f4 type; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Row of the 16 x 16 result that element i of lane-group kq (= lane / 16) holds.
template <typename real>
__device__ __forceinline__ constexpr int drow(int i, int kq) { return sizeof(real) == 8 ? 4 * i + kq : 4 * kq + i; }

// Waves per workgroup (one 16-element tile each): fewer for large Np, whose R tiles fill LDS.
template <int NP>
constexpr int waves_for() { return NP <= 128 ? 4 : 1; }

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename real, int NP, int kWaves = waves_for<NP>()>
__global__ __launch_bounds__(64 * kWaves) void wadg_dense_kernel(DenseArgs<real> a) {
  typedef typename Acc4<real>::type v4;
  constexpr int NPP = (NP + 15) / 16 * 16;  // coefficients padded to the tile size
  constexpr int NT = NPP / 16, NK = NPP / 4;
  __shared__ real rt[kWaves][NPP][16];   // R tile, coefficient-major
  __shared__ real ut[kWaves][16][16];    // U chunk, point-major
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t k0 = ((int64_t)blockIdx.x * kWaves + wave) * 16;
  if (k0 >= a.K) return;  // waves only synchronise among their own lanes
  for (int idx = lane; idx < NPP * 16; idx += 64) {
    const int i = idx >> 4, e = idx & 15;
    rt[wave][i][e] = (i < NP && k0 + e < a.K) ? a.r[(size_t)(k0 + e) * NP + i] : real(0);
  }
  wsync();
  v4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4{0, 0, 0, 0};
  const int64_t ke = k0 + col < a.K ? k0 + col : a.K - 1;  // stand-in element for the tail
  const real* c2e = a.c2q + (size_t)ke * a.nqp;
  for (int qc = 0; qc < a.nqc; ++qc) {
    const real* va = a.va + (size_t)qc * NK * 64 + lane;
    v4 u = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) u = mfma(va[ks * 64], rt[wave][4 * ks + kq][col], u);
    const real* cq = c2e + qc * 16;  // c^2 at the chunk's points
#pragma unroll
    for (int i = 0; i < 4; ++i) ut[wave][drow<real>(i, kq)][col] = u[i] * cq[drow<real>(i, kq)];
    wsync();
    const real* pa = a.pa + (size_t)qc * NT * 4 * 64 + lane;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc[t] = mfma(pa[(t * 4 + ks) * 64], ut[wave][4 * ks + kq][col], acc[t]);
    wsync();  // the next chunk overwrites ut
  }
  if (k0 + col < a.K) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = t * 16 + drow<real>(i, kq);
        if (row < NP) a.out[(size_t)(k0 + col) * NP + row] = acc[t][i];
      }
  }
}

template <typename real, int NP>
int launch_typed(const DenseArgs<real>& a, void* stream) {
  constexpr int kWaves = waves_for<NP>();
  const int64_t tiles = (a.K + 15) / 16;
  const int64_t blocks = (tiles + kWaves - 1) / kWaves;
  hipLaunchKernelGGL((wadg_dense_kernel<real, NP>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace

template <typename real>
int launch_wadg_dense(int N, const DenseArgs<real>& a, void* stream) {
  if (a.K <= 0) return 0;
  switch (N) {
    case 1: return launch_typed<real, dimp(1)>(a, stream);
    case 2: return launch_typed<real, dimp(2)>(a, stream);
    case 3: return launch_typed<real, dimp(3)>(a, stream);
    case 4: return launch_typed<real, dimp(4)>(a, stream);
    case 5: return launch_typed<real, dimp(5)>(a, stream);
    case 6: return launch_typed<real, dimp(6)>(a, stream);
    case 7: return launch_typed<real, dimp(7)>(a, stream);
    case 8: return launch_typed<real, dimp(8)>(a, stream);
    case 9: return launch_typed<real, dimp(9)>(a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template int launch_wadg_dense<double>(int, const DenseArgs<double>&, void*);
template int launch_wadg_dense<float>(int, const DenseArgs<float>&, void*);

}  // namespace bbw
