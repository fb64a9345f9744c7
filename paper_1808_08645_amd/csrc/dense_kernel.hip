// Dense quadrature WADG update (paper Section 3.3, eq. pwadg) on the matrix cores (FP64, or
// FP32 with FP32 accumulation):
//     out = P_q diag(c^2(x_q)) V_q r
// per element, with V_q the Bernstein basis at the Nq points of a collapsed Gauss-Jacobi
// rule and P_q = M^{-1} V_q^T W the quadrature L^2 projection. It is the comparison
// baseline of the fast Bernstein update: O(Nq Np) = O(N^6) work per element instead of
// O(N^4), and Nq values of c^2 stored per element instead of Mp coefficients.
//
// Both products are dense contractions shared by all elements, so a tile of 16 elements
// runs them on v_mfma_f64_16x16x4f64 (v_mfma_f32_16x16x4f32):
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

// A workgroup of kW waves owns one tile of 16 elements; R is staged once in LDS for all of
// them. The point chunks go in groups of kW: in a group, wave w forms U for chunk
// group * kW + w (its own first product) and writes U * c^2 to LDS; after one barrier, every
// wave adds the contributions of all kW chunks to its share of the output tiles (tiles
// w, w + kW, ...). Per tile and chunk the MFMAs are those of one wave doing both products,
// but the R tile and the accumulators are split kW ways, so several waves per SIMD fit
// where a wave per tile would hold a whole R tile in LDS (N >= 8) and every accumulator in
// registers. U is double-buffered across groups, which leaves one barrier per group. Small
// elements have fewer output tiles than 4: then as many waves as tiles.
template <int NP>
constexpr int dense_waves() {
  return (NP + 15) / 16 < 4 ? (NP + 15) / 16 : 4;
}

template <typename real, int NP, int kW = dense_waves<NP>()>
__global__ __launch_bounds__(64 * kW)
void wadg_dense_kernel(DenseArgs<real> a) {
  typedef typename Acc4<real>::type v4;
  constexpr int NPP = (NP + 15) / 16 * 16;  // coefficients padded to the tile size
  constexpr int NT = NPP / 16, NK = NPP / 4;
  constexpr int TPW = (NT + kW - 1) / kW;   // output tiles per wave
  __shared__ real rt[NPP][16];              // R tile, coefficient-major
  __shared__ real ut[2][kW][16][16];        // U * c^2 of the group's chunks, point-major
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * 16;
  for (int idx = threadIdx.x; idx < NPP * 16; idx += 64 * kW) {
    const int i = idx >> 4, e = idx & 15;
    rt[i][e] = (i < NP && k0 + e < a.K) ? a.r[(size_t)(k0 + e) * NP + i] : real(0);
  }
  __syncthreads();
  v4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = v4{0, 0, 0, 0};
  const int64_t ke = k0 + col < a.K ? k0 + col : a.K - 1;  // stand-in element for the tail
  const real* c2e = a.c2q + (size_t)ke * a.nqp;
  const int ngroups = (a.nqc + kW - 1) / kW;
  for (int g = 0; g < ngroups; ++g) {
    const int buf = g & 1;
    const int qc = g * kW + wave;
    if (qc < a.nqc) {  // uniform per wave
      const real* va = a.va + (size_t)qc * NK * 64 + lane;
      v4 u0 = {0, 0, 0, 0}, u1 = {0, 0, 0, 0};  // two chains: consecutive MFMAs independent
#pragma unroll
      for (int ks = 0; ks < NK; ks += 2) {
        u0 = mfma(va[ks * 64], rt[4 * ks + kq][col], u0);
        if (ks + 1 < NK) u1 = mfma(va[(ks + 1) * 64], rt[4 * ks + 4 + kq][col], u1);
      }
      const real* cq = c2e + qc * 16;  // c^2 at the chunk's points
#pragma unroll
      for (int i = 0; i < 4; ++i) ut[buf][wave][drow<real>(i, kq)][col] = (u0[i] + u1[i]) * cq[drow<real>(i, kq)];
    }
    __syncthreads();  // the group's U are written; the group before last is read by all
#pragma unroll
    for (int w2 = 0; w2 < kW; ++w2) {
      const int qc2 = g * kW + w2;
      if (qc2 < a.nqc) {  // uniform
        const real* pa = a.pa + (size_t)qc2 * NT * 4 * 64 + lane;
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
          const int t = wave + kW * tt;
          if (t < NT) {  // uniform per wave
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
              acc[tt] = mfma(pa[(t * 4 + ks) * 64], ut[buf][w2][4 * ks + kq][col], acc[tt]);
          }
        }
      }
    }
  }
  if (k0 + col < a.K) {
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int t = wave + kW * tt;
      if (t < NT) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = t * 16 + drow<real>(i, kq);
          if (row < NP) a.out[(size_t)(k0 + col) * NP + row] = acc[tt][i];
        }
      }
    }
  }
}

template <typename real, int NP>
int launch_typed(const DenseArgs<real>& a, void* stream) {
  const int64_t tiles = (a.K + 15) / 16;
  hipLaunchKernelGGL((wadg_dense_kernel<real, NP>), dim3((unsigned)tiles), dim3(64 * dense_waves<NP>()), 0,
                     (hipStream_t)stream, a);
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
