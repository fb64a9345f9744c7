// Dense quadrature WADG update (paper Section 3.3, eq. pwadg) on the FP64 matrix cores:
//     out = P_q diag(c^2(x_q)) V_q r
// per element, with V_q the Bernstein basis at the Nq points of a collapsed Gauss-Jacobi
// rule and P_q = M^{-1} V_q^T W the quadrature L^2 projection. It is the comparison
// baseline of the fast Bernstein update: O(Nq Np) = O(N^6) work per element instead of
// O(N^4), and Nq values of c^2 stored per element instead of Mp coefficients.
//
// Both products are dense contractions shared by all elements, so a wavefront takes a
// tile of 16 elements and runs them on v_mfma_f64_16x16x4f64:
//   U (16 points x 16 elements) = V_q[chunk] (16 x Np) . R (Np x 16)       Np/4 MFMAs
//   U *= c^2 at those points (per element)
//   Out (Np x 16) += P_q[:, chunk] (Np x 16) . U (16 x 16)                  Np/4 MFMAs
// over the point chunks. The tables are stored in the MFMA operand order (one coalesced
// 512-byte load per operand, L2-resident); R and U pass through LDS to change from the
// accumulator layout to the B-operand layout. Lane l holds A[l%16][l/16], B[l/16][l%16]
// and D[4i + l/16][l%16] as element i = 0..3 of its result (checked on the device).
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Waves per workgroup (one 16-element tile each): fewer for large Np, whose R tiles fill LDS.
template <int NP>
constexpr int waves_for() { return NP <= 128 ? 4 : 1; }

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NP, int kWaves = waves_for<NP>()>
__global__ __launch_bounds__(64 * kWaves) void wadg_dense_kernel(DenseArgs a) {
  constexpr int NPP = (NP + 15) / 16 * 16;  // coefficients padded to the tile size
  constexpr int NT = NPP / 16, NK = NPP / 4;
  __shared__ double rt[kWaves][NPP][16];   // R tile, coefficient-major
  __shared__ double ut[kWaves][16][16];    // U chunk, point-major
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t k0 = ((int64_t)blockIdx.x * kWaves + wave) * 16;
  if (k0 >= a.K) return;  // waves only synchronise among their own lanes
  for (int idx = lane; idx < NPP * 16; idx += 64) {
    const int i = idx >> 4, e = idx & 15;
    rt[wave][i][e] = (i < NP && k0 + e < a.K) ? a.r[(size_t)(k0 + e) * NP + i] : 0.0;
  }
  wsync();
  d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t ke = k0 + col < a.K ? k0 + col : a.K - 1;  // stand-in element for the tail
  const double* c2e = a.c2q + (size_t)ke * a.nqp + kq;  // point 16 qc + 4 i + kq
  for (int qc = 0; qc < a.nqc; ++qc) {
    const double* va = a.va + (size_t)qc * NK * 64 + lane;
    d4 u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) u = __builtin_amdgcn_mfma_f64_16x16x4f64(va[ks * 64], rt[wave][4 * ks + kq][col], u, 0, 0, 0);
    const double* cq = c2e + qc * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) ut[wave][4 * i + kq][col] = u[i] * cq[4 * i];
    wsync();
    const double* pa = a.pa + (size_t)qc * NT * 4 * 64 + lane;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[(t * 4 + ks) * 64], ut[wave][4 * ks + kq][col], acc[t], 0, 0, 0);
    wsync();  // the next chunk overwrites ut
  }
  if (k0 + col < a.K) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = t * 16 + 4 * i + kq;
        if (row < NP) a.out[(size_t)(k0 + col) * NP + row] = acc[t][i];
      }
  }
}

template <int NP>
int launch_typed(const DenseArgs& a, void* stream) {
  constexpr int kWaves = waves_for<NP>();
  const int64_t tiles = (a.K + 15) / 16;
  const int64_t blocks = (tiles + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(wadg_dense_kernel<NP>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace

int launch_wadg_dense(int N, const DenseArgs& a, void* stream) {
  if (a.K <= 0) return 0;
  switch (N) {
    case 1: return launch_typed<dimp(1)>(a, stream);
    case 2: return launch_typed<dimp(2)>(a, stream);
    case 3: return launch_typed<dimp(3)>(a, stream);
    case 4: return launch_typed<dimp(4)>(a, stream);
    case 5: return launch_typed<dimp(5)>(a, stream);
    case 6: return launch_typed<dimp(6)>(a, stream);
    case 7: return launch_typed<dimp(7)>(a, stream);
    case 8: return launch_typed<dimp(8)>(a, stream);
    case 9: return launch_typed<dimp(9)>(a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace bbw
