// Kernels of the receiver misfit and its adjoint (gradient with respect to c^2_M).
//
// The adjoint recursion itself runs on the stage kernel (see host.cpp): with the velocity
// reflection S = diag(1, -1, -1, -1) and the block mass matrix M, the transposed DG-WADG
// operator satisfies A^T (M S) = (M S) (B W), so in the variables z = (M S)^{-1} lambda every
// transposed stage is a plain-DG right-hand side B applied after the weight adjustment W.
// What is left for this file is elementwise and small:
//   * lincomb      x = alpha x + beta y (the 2N-storage bookkeeping of the reversed stages);
//   * sample       pressure at the receivers, p(x_r) = sum_a q_p[k_r][a] B_a(x_r), in FP64;
//   * inject       z_p[k_r] += resid_r (J_k M)^{-1} b_r (dJ/dq mapped into z);
//   * c2grad       grad[k][g] += scale J_k sum_q w_q B^M_g(x_q) y(x_q) v(x_q): the derivative
//                  of v^T M^{-1} M_{c^2} y with respect to the Bernstein coefficients of c^2_M.
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

template <typename real>
__global__ __launch_bounds__(256) void lincomb_kernel(real* x, const real* y, real alpha, real beta, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = alpha * x[i] + beta * y[i];
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

// One workgroup of 256 threads per element; each thread owns rule points q = tid + 256 i.
// vt[a][q] = B^N_a(x_q) and bw[q][g] = w_q B^M_g(x_q) (rule of degree >= 2N + M).
constexpr int kGradThreads = 256;

template <typename real>
__global__ __launch_bounds__(kGradThreads) void c2grad_kernel(C2GradArgs<real> a) {
  __shared__ double ys[256], vs[256];  // Np <= 220
  __shared__ double red[kGradThreads / 64][16];
  const int64_t k = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < a.Np; i += kGradThreads) {
    ys[i] = (double)a.y[(size_t)k * a.Np + i];
    vs[i] = (double)a.v[(size_t)k * a.Np + i];
  }
  __syncthreads();
  double part[16];
#pragma unroll
  for (int g = 0; g < 16; ++g) part[g] = 0.0;
  for (int q = tid; q < a.nq; q += kGradThreads) {
    double yq = 0.0, vq = 0.0;
    for (int i = 0; i < a.Np; ++i) {
      const double b = a.vt[(size_t)i * a.nq + q];
      yq += b * ys[i];
      vq += b * vs[i];
    }
    const double pr = yq * vq;
#pragma unroll
    for (int g = 0; g < 16; ++g)
      if (g < a.Mp) part[g] += a.bw[(size_t)q * a.Mp + g] * pr;
  }
#pragma unroll
  for (int g = 0; g < 16; ++g) {
    double s = part[g];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave][g] = s;
  }
  __syncthreads();
  if (tid < a.Mp) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kGradThreads / 64; ++w) s += red[w][tid];
    a.grad[(size_t)k * a.Mp + tid] += a.scale * a.J[k] * s;
  }
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
int launch_c2grad(const C2GradArgs<real>& a, void* stream) {
  if (a.K <= 0) return 0;
  if (a.Np > 256 || a.Mp > 16) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(c2grad_kernel<real>, dim3((unsigned)a.K), dim3(kGradThreads), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

template int launch_lincomb<double>(double*, const double*, double, double, int64_t, void*);
template int launch_lincomb<float>(float*, const float*, double, double, int64_t, void*);
template int launch_sample<double>(const double*, const int32_t*, const double*, int32_t, int32_t, double*, void*);
template int launch_sample<float>(const float*, const int32_t*, const double*, int32_t, int32_t, double*, void*);
template int launch_inject<double>(double*, const int32_t*, const double*, const double*, int32_t, int32_t, void*);
template int launch_inject<float>(float*, const int32_t*, const double*, const double*, int32_t, int32_t, void*);
template int launch_c2grad<double>(const C2GradArgs<double>&, void*);
template int launch_c2grad<float>(const C2GradArgs<float>&, void*);

}  // namespace bbw
