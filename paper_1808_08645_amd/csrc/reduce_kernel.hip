// FP64 quadrature reductions of a state (off the time-step path): the squared L^2 error
// against sampled values of a reference solution, and the acoustic energy
//     E = 1/2 sum_k J_k int_ref ( p^2 / c^2_M + |u|^2 )
// of the system (1/c^2) p_t + div u = 0, u_t + grad p = 0 (paper Section 3.1).
//
// Both evaluate the Bernstein expansion of every field at the points of one collapsed
// Gauss-Jacobi rule per element: values = Q B^T, a contraction of (4 K) x Np by Np x nq.
// A group of kRedElems elements is staged in LDS (FP64, coefficient-major so that one
// coefficient of all fields of the group is one contiguous run) and each thread owns one
// rule point: it streams the point's column of the basis table (coalesced over points,
// L2-resident) and updates 4 kRedElems accumulators per table entry. Squares, weights and
// the division by c^2_M are applied in registers; only per-block partial sums leave the
// kernel and the host adds them in a fixed order, so the result is deterministic.
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedElems = 8;
constexpr int kRedSlots = kRedElems * 4;

template <typename real, int MODE>
__global__ __launch_bounds__(kRedThreads) void quad_reduce_kernel(QuadReduceArgs a) {
  extern __shared__ double lds[];
  const int Np = a.Np, Mp = a.Mp, nq = a.nq;
  double* sq = lds;                         // [Np][kRedElems][4]
  double* sc = sq + (size_t)Np * kRedSlots;  // [Mp][kRedElems]
  double* red = sc + (size_t)Mp * kRedElems;  // [kRedThreads / 64][4]
  const real* q = static_cast<const real*>(a.q);
  const real* c2 = static_cast<const real*>(a.c2);
  const int64_t nk = a.k1 - a.k0;
  const int64_t ngroups = (nk + kRedElems - 1) / kRedElems;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};

  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int64_t kb = a.k0 + g * kRedElems;  // first element of the group
    const int ne = (int)((a.k1 - kb) < kRedElems ? (a.k1 - kb) : kRedElems);
    __syncthreads();  // the previous group's LDS reads are complete
    for (int i = threadIdx.x; i < Np * kRedSlots; i += kRedThreads) {
      const int j = i / kRedSlots, r = i - j * kRedSlots, e = r >> 2, f = r & 3;
      sq[i] = e < ne ? (double)q[((size_t)f * a.K + (size_t)(kb + e)) * Np + j] : 0.0;
    }
    if (MODE == 1)
      for (int i = threadIdx.x; i < Mp * kRedElems; i += kRedThreads) {
        const int j = i / kRedElems, e = i - j * kRedElems;
        sc[i] = e < ne ? (double)c2[(size_t)(kb + e) * Mp + j] : 1.0;
      }
    __syncthreads();
    for (int p = threadIdx.x; p < nq; p += kRedThreads) {
      double v[kRedSlots];
#pragma unroll
      for (int s = 0; s < kRedSlots; ++s) v[s] = 0.0;
      for (int j = 0; j < Np; ++j) {
        const double b = a.basis[(size_t)j * nq + p];
        const double* row = sq + (size_t)j * kRedSlots;
#pragma unroll
        for (int s = 0; s < kRedSlots; ++s) v[s] += b * row[s];
      }
      const double wp = a.w[p];
      if (MODE == 0) {
#pragma unroll
        for (int e = 0; e < kRedElems; ++e) {
          if (e < ne) {
            const double wj = wp * a.J[kb + e];
            const size_t ke = (size_t)(kb - a.k0 + e);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
              const double d = v[4 * e + f] - a.exact[((size_t)f * nk + ke) * nq + p];
              acc[f] += wj * d * d;
            }
          }
        }
      } else {
        double cv[kRedElems];
#pragma unroll
        for (int e = 0; e < kRedElems; ++e) cv[e] = 0.0;
        for (int j = 0; j < Mp; ++j) {
          const double b = a.basis_c2[(size_t)j * nq + p];
#pragma unroll
          for (int e = 0; e < kRedElems; ++e) cv[e] += b * sc[j * kRedElems + e];
        }
#pragma unroll
        for (int e = 0; e < kRedElems; ++e) {
          if (e < ne) {
            const double hw = 0.5 * wp * a.J[kb + e];
            acc[0] += hw * v[4 * e] * v[4 * e] / cv[e];
#pragma unroll
            for (int f = 1; f < 4; ++f) acc[f] += hw * v[4 * e + f] * v[4 * e + f];
          }
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double x = acc[f];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) red[wave * 4 + f] = x;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += red[w * 4 + threadIdx.x];
    a.partial[(size_t)blockIdx.x * 4 + threadIdx.x] = s;
  }
}

template <typename real, int MODE>
int launch_typed(const QuadReduceArgs& a, int nblocks, void* stream) {
  const size_t shmem = ((size_t)a.Np * kRedSlots + (size_t)a.Mp * kRedElems + 4 * (kRedThreads / 64)) * 8;
  hipLaunchKernelGGL((quad_reduce_kernel<real, MODE>), dim3(nblocks), dim3(kRedThreads), shmem,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace

int quad_reduce_blocks(int64_t nelems, int max_blocks) {
  const int64_t groups = (nelems + kRedElems - 1) / kRedElems;
  return (int)(groups < max_blocks ? (groups > 0 ? groups : 1) : max_blocks);
}

int launch_quad_reduce(int dtype, int mode, const QuadReduceArgs& a, int nblocks, void* stream) {
  if (a.Np > dimp(kMaxN) || a.Mp > dimp(kMaxM) || a.nq <= 0 || nblocks <= 0) return (int)hipErrorInvalidValue;
  if (dtype == 0) return mode == 0 ? launch_typed<double, 0>(a, nblocks, stream) : launch_typed<double, 1>(a, nblocks, stream);
  return mode == 0 ? launch_typed<float, 0>(a, nblocks, stream) : launch_typed<float, 1>(a, nblocks, stream);
}

}  // namespace bbw
