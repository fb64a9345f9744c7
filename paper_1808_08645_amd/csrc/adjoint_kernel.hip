// Kernels of the receiver misfit and its adjoint (gradient with respect to c^2_M).
//
// The adjoint recursion itself runs on the stage kernel (see host.cpp): with the velocity
// reflection S = diag(1, -1, -1, -1) and the block mass matrix M, the transposed DG-WADG
// operator satisfies A^T (M S) = (M S) (B W), so in the variables z = (M S)^{-1} lambda every
// transposed stage is a plain-DG right-hand side B applied after the weight adjustment W.
// What is left for this file is elementwise and small:
//   * lincomb, back_update   the 2N-storage bookkeeping of the reversed stages;
//   * sample       pressure at the receivers, p(x_r) = sum_a q_p[k_r][a] B_a(x_r), in FP64;
//   * inject       z_p[k_r] += resid_r (J_k M)^{-1} b_r (dJ/dq mapped into z);
//   * c2grad       grad[k][g] += scale J_k sum_q w_q B^M_g(x_q) y(x_q) v(x_q): the derivative
//                  of v^T M^{-1} M_{c^2} y with respect to the Bernstein coefficients of c^2_M,
//                  a dense contraction per element, on the FP64 matrix cores.
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

template <typename real>
__global__ __launch_bounds__(256) void lincomb_kernel(real* x, const real* y, real alpha, real beta, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = alpha * x[i] + beta * y[i];
}

// One reversed stage's bookkeeping in one pass: z_q += dt t, then (if v_coef) v = a v + b z_q.
template <typename real>
__global__ __launch_bounds__(256) void back_update_kernel(real* zq, real* v, const real* t, real dt, real a, real b,
                                                          int v_coef, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const real z = zq[i] + dt * t[i];
    zq[i] = z;
    if (v_coef) v[i] = a * v[i] + b * z;
  }
}

// One wavefront per receiver.
template <typename real>
__global__ __launch_bounds__(64) void sample_kernel(const real* qp, const int32_t* elem, const double* basis, int32_t nrec,
                                                    int32_t Np, double* out) {
  const int r = blockIdx.x, lane = threadIdx.x;
  if (r >= nrec) return;
  const real* q = qp + (size_t)elem[r] * Np;
  const double* b = basis + (size_t)r * Np;
  double s = 0.0;
  for (int a = lane; a < Np; a += 64) s += (double)q[a] * b[a];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[r] = s;
}

// One workgroup; receivers in sequence, coefficient a always handled by the same thread, so
// receivers that share an element update each coefficient in order without races.
template <typename real>
__global__ __launch_bounds__(256) void inject_kernel(real* zp, const int32_t* elem, const double* kvec,
                                                     const double* resid, int32_t nrec, int32_t Np) {
  for (int r = 0; r < nrec; ++r) {
    const double c = resid[r];
    real* z = zp + (size_t)elem[r] * Np;
    const double* kv = kvec + (size_t)r * Np;
    for (int a = threadIdx.x; a < Np; a += blockDim.x) z[a] = (real)((double)z[a] + c * kv[a]);
  }
}

// grad[k][g] += scale J_k sum_q w_q B^M_g(x_q) y_k(x_q) v_k(x_q) on the FP64 matrix cores,
// with the tiling of the dense WADG kernel: a wavefront takes 16 elements; per chunk of 16
// rule points it forms Y = V_q R_y and V = V_q R_v (the two products share every A operand),
// multiplies them pointwise, and accumulates G (16 x 16 elements) += BW^T[:, chunk] (Y.V),
// where BW^T holds w_q B^M_g(x_q) in rows g < Mp. Lane l holds A[l%16][l/16], B[l/16][l%16]
// and D[4i + l/16][l%16] as element i of its result.
typedef double d4 __attribute__((ext_vector_type(4)));

template <int NP>
constexpr int grad_waves() {
  constexpr int NPP = (NP + 15) / 16 * 16;
  constexpr int per_wave = (2 * NPP * 16 + 16 * 16) * 8;  // two coefficient tiles and the product
  return 61440 / per_wave >= 4 ? 4 : (61440 / per_wave >= 1 ? 61440 / per_wave : 1);
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename real, int NP, int kWaves = grad_waves<NP>()>
__global__ __launch_bounds__(64 * kWaves) void c2grad_kernel(C2GradArgs<real> a) {
  constexpr int NPP = (NP + 15) / 16 * 16, NK = NPP / 4;
  __shared__ double ry[kWaves][NPP][16], rv[kWaves][NPP][16], pt[kWaves][16][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t k0 = ((int64_t)blockIdx.x * kWaves + wave) * 16;
  if (k0 >= a.K) return;  // waves only synchronise among their own lanes
  for (int idx = lane; idx < NPP * 16; idx += 64) {
    const int i = idx >> 4, e = idx & 15;
    const bool ok = i < NP && k0 + e < a.K;
    ry[wave][i][e] = ok ? (double)a.y[(size_t)(k0 + e) * NP + i] : 0.0;
    rv[wave][i][e] = ok ? (double)a.v[(size_t)(k0 + e) * NP + i] : 0.0;
  }
  wsync();
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int qc = 0; qc < a.nqc; ++qc) {
    const double* va = a.va + (size_t)qc * NK * 64 + lane;
    d4 uy = {0.0, 0.0, 0.0, 0.0}, uv = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
      const double A = va[ks * 64];
      uy = __builtin_amdgcn_mfma_f64_16x16x4f64(A, ry[wave][4 * ks + kq][col], uy, 0, 0, 0);
      uv = __builtin_amdgcn_mfma_f64_16x16x4f64(A, rv[wave][4 * ks + kq][col], uv, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) pt[wave][4 * i + kq][col] = uy[i] * uv[i];
    wsync();
    const double* bw = a.bwa + (size_t)qc * 4 * 64 + lane;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bw[ks * 64], pt[wave][4 * ks + kq][col], acc, 0, 0, 0);
    wsync();  // the next chunk overwrites pt
  }
  if (k0 + col < a.K) {
    const double f = a.scale * a.J[k0 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int g = 4 * i + kq;
      if (g < a.Mp) a.grad[(size_t)(k0 + col) * a.Mp + g] += f * acc[i];
    }
  }
}

template <typename real, int NP>
int launch_grad_typed(const C2GradArgs<real>& a, void* stream) {
  constexpr int kWaves = grad_waves<NP>();
  const int64_t tiles = (a.K + 15) / 16;
  const int64_t blocks = (tiles + kWaves - 1) / kWaves;
  hipLaunchKernelGGL((c2grad_kernel<real, NP>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

template <typename real>
int launch_lincomb(real* x, const real* y, double alpha, double beta, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(lincomb_kernel<real>, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, (real)alpha,
                     (real)beta, n);
  return (int)hipGetLastError();
}

template <typename real>
int launch_back_update(real* zq, real* v, const real* t, double dt, double a, double b, bool update_v, int64_t n,
                       void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(back_update_kernel<real>, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, zq, v, t, (real)dt,
                     (real)a, (real)b, update_v ? 1 : 0, n);
  return (int)hipGetLastError();
}

template <typename real>
int launch_sample(const real* qp, const int32_t* elem, const double* basis, int32_t nrec, int32_t Np, double* out,
                  void* stream) {
  if (nrec <= 0) return 0;
  hipLaunchKernelGGL(sample_kernel<real>, dim3(nrec), dim3(64), 0, (hipStream_t)stream, qp, elem, basis, nrec, Np, out);
  return (int)hipGetLastError();
}

template <typename real>
int launch_inject(real* zp, const int32_t* elem, const double* kvec, const double* resid, int32_t nrec, int32_t Np,
                  void* stream) {
  if (nrec <= 0) return 0;
  hipLaunchKernelGGL(inject_kernel<real>, dim3(1), dim3(256), 0, (hipStream_t)stream, zp, elem, kvec, resid, nrec, Np);
  return (int)hipGetLastError();
}

template <typename real>
int launch_c2grad(int N, const C2GradArgs<real>& a, void* stream) {
  if (a.K <= 0) return 0;
  if (a.Mp > 16) return (int)hipErrorInvalidValue;
  switch (N) {
    case 1: return launch_grad_typed<real, dimp(1)>(a, stream);
    case 2: return launch_grad_typed<real, dimp(2)>(a, stream);
    case 3: return launch_grad_typed<real, dimp(3)>(a, stream);
    case 4: return launch_grad_typed<real, dimp(4)>(a, stream);
    case 5: return launch_grad_typed<real, dimp(5)>(a, stream);
    case 6: return launch_grad_typed<real, dimp(6)>(a, stream);
    case 7: return launch_grad_typed<real, dimp(7)>(a, stream);
    case 8: return launch_grad_typed<real, dimp(8)>(a, stream);
    case 9: return launch_grad_typed<real, dimp(9)>(a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template int launch_lincomb<double>(double*, const double*, double, double, int64_t, void*);
template int launch_lincomb<float>(float*, const float*, double, double, int64_t, void*);
template int launch_back_update<double>(double*, double*, const double*, double, double, double, bool, int64_t, void*);
template int launch_back_update<float>(float*, float*, const float*, double, double, double, bool, int64_t, void*);
template int launch_sample<double>(const double*, const int32_t*, const double*, int32_t, int32_t, double*, void*);
template int launch_sample<float>(const float*, const int32_t*, const double*, int32_t, int32_t, double*, void*);
template int launch_inject<double>(double*, const int32_t*, const double*, const double*, int32_t, int32_t, void*);
template int launch_inject<float>(float*, const int32_t*, const double*, const double*, int32_t, int32_t, void*);
template int launch_c2grad<double>(int, const C2GradArgs<double>&, void*);
template int launch_c2grad<float>(int, const C2GradArgs<float>&, void*);

}  // namespace bbw
