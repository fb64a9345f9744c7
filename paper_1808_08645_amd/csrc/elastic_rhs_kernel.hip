// DG right-hand side of the elastic velocity-stress system before the weight adjustment
// (paper Section 2.2, the semi-discrete form after eq. ewave), isotropic or not (the media
// enter only through the weight-adjusted update that follows):
//   r_v = sum_i A_i^T d sigma/dx_i + sum_f Fscale_f L^f F_v,  F_v = A_n^T [[sigma]]/2 + tau_v A_n^T A_n [[v]]/2
//   r_s = sum_i A_i  d v/dx_i      + sum_f Fscale_f L^f F_s,  F_s = A_n [[v]]/2 + tau_s A_n A_n^T [[sigma]]/2
// Fields v1, v2, v3, sigma xx, yy, zz, yz, xz, xy (Voigt order).
//
// One wavefront per element (grid-stride), in its LDS slice:
//  * volume: Bernstein derivative stencils at degree N-1, d/dr_j f -> (N/2)(f_{g+e_j} - f_{g+e_0}),
//    combined with G = dr/dx into the 9 outputs, then elevated to degree N;
//  * fluxes on the face coefficients (the trace of a Bernstein polynomial on a face is the 2D
//    Bernstein polynomial of the coefficients with alpha_f = 0), neighbour coefficients read at the
//    same face multi-index (element vertices are stored in ascending order, so a shared face lists
//    its vertices in the same order on both sides), mirror states on walls;
//  * lift: L^f = M^{-1} M_f as a dense Bernstein matrix per reference face (a first version;
//    the acoustic kernel uses the sparse factorisation of Section 4).
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename real, int N>
struct ElRhsLayout {
  static constexpr int NP = dimp(N), NQ = dimp(N - 1), NFP = dim2(N);
  static constexpr int OFF_Q = 0, OFF_D = 9 * NP, OFF_R = OFF_D + 9 * NQ, OFF_F = OFF_R + 9 * NP,
                       TOTAL = OFF_F + 4 * 9 * NFP;
  static constexpr int TABLES = 16 * NP + 4 * 4 * NFP;
  static constexpr int per = TOTAL * (int)sizeof(real);
  static constexpr int WAVES = (61440 - TABLES) / per >= 4 ? 4 : ((61440 - TABLES) / per >= 1 ? (61440 - TABLES) / per : 1);
};

template <typename real, int N>
__global__ __launch_bounds__((64 * ElRhsLayout<real, N>::WAVES)) void elastic_rhs_kernel(ElasticRhsArgs<real> a) {
  using L = ElRhsLayout<real, N>;
  constexpr int NP = L::NP, NQ = L::NQ, NFP = L::NFP, WPB = L::WAVES;
  __shared__ real smem[WPB * L::TOTAL];
  __shared__ uint4 itab[NP];
  __shared__ int fpos[4 * NFP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  real* const Qs = smem + wave * L::TOTAL + L::OFF_Q;
  real* const Dn = smem + wave * L::TOTAL + L::OFF_D;
  real* const Rs = smem + wave * L::TOTAL + L::OFF_R;
  real* const Fs = smem + wave * L::TOTAL + L::OFF_F;

  // itab[i] for the multi-index a at graded position i (s = |a|, D(s) = (s+1)(s+2)/2):
  //   x: pos(a+e1) | pos(a+e3) << 16 (pos(a+e2) = pos(a+e1) + 1); y: pos(a-e1) | pos(a-e2) << 16;
  //   z: pos(a-e3) | a1 << 16 | a2 << 24; w: a3 | s << 8  (pos(a-e_j) = 0 where a_j = 0)
  for (int i = threadIdx.x; i < NP; i += 64 * WPB) {
    int d = 0;
    while (d < N && dimp(d) <= i) ++d;
    int r = i - dimp(d - 1), a3 = 0;
    while (a3 < d && r >= d + 1 - a3) r -= d + 1 - a3, ++a3;
    const int a2 = r, a1 = d - a3 - r;
    const int du = (d + 1) * (d + 2) / 2, dd = d * (d + 1) / 2;
    uint4 t;
    t.x = (uint32_t)(i + du + a3) | ((uint32_t)(i + du + d + 2) << 16);
    t.y = (uint32_t)(a1 > 0 ? i - dd - a3 : 0) | ((uint32_t)(a2 > 0 ? i - dd - a3 - 1 : 0) << 16);
    t.z = (uint32_t)(a3 > 0 ? i - dd - d - 1 : 0) | ((uint32_t)a1 << 16) | ((uint32_t)a2 << 24);
    t.w = (uint32_t)a3 | ((uint32_t)d << 8);
    itab[i] = t;
  }
  for (int i = threadIdx.x; i < 4 * NFP; i += 64 * WPB) fpos[i] = a.fpos[i];
  __syncthreads();

  // the terms of the 9 outputs: (field, direction) pairs, up to 3 per output
  // v1: sxx/x + sxy/y + sxz/z; v2: sxy/x + syy/y + syz/z; v3: sxz/x + syz/y + szz/z;
  // sxx: v1/x; syy: v2/y; szz: v3/z; syz: v3/y + v2/z; sxz: v3/x + v1/z; sxy: v2/x + v1/y
  constexpr int tf[9][3] = {{3, 8, 7}, {8, 4, 6}, {7, 6, 5}, {0, -1, -1}, {1, -1, -1}, {2, -1, -1},
                            {2, 1, -1}, {2, 0, -1}, {1, 0, -1}};
  constexpr int td[9][3] = {{0, 1, 2}, {0, 1, 2}, {0, 1, 2}, {0, 0, 0}, {1, 0, 0}, {2, 0, 0},
                            {1, 2, 0}, {0, 2, 0}, {0, 1, 0}};
  const real halfN = real(N) / real(2);
  const int64_t K = a.K;
  for (int64_t k = (int64_t)blockIdx.x * WPB + wave; k < K; k += (int64_t)gridDim.x * WPB) {
    for (int t = lane; t < 9 * NP; t += 64) {
      const int f = t / NP, i = t - f * NP;
      Qs[f * NP + i] = a.q[((size_t)f * K + k) * NP + i];
    }
    const real* geo = a.geo + (size_t)k * kGeoStride;
    real G[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) G[j] = geo[j];  // G[3i + j] = d r_j / d x_i
    wsync();
    // volume at degree N - 1: sum over terms of sum_j G[dir][j] (N/2)(f_{g+e_j} - f_g)
    for (int t = lane; t < 9 * NQ; t += 64) {
      const int c = t / NQ, g = t - c * NQ;
      const uint4 e = itab[g];
      const int u1 = e.x & 0xFFFF, u3 = e.x >> 16;
      real d = real(0);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int fd = tf[c][m];
        if (fd < 0) continue;
        const int dir = td[c][m];
        const real* fq = Qs + fd * NP;
        const real f0 = fq[g];
        d += G[3 * dir + 0] * (fq[u1] - f0) + G[3 * dir + 1] * (fq[u1 + 1] - f0) + G[3 * dir + 2] * (fq[u3] - f0);
      }
      Dn[c * NQ + g] = halfN * d;
    }
    wsync();
    // elevation to degree N: (E y)_a = sum_{j: a_j > 0} (a_j / N) y_{a - e_j}
    for (int t = lane; t < 9 * NP; t += 64) {
      const int c = t / NP, i = t - c * NP;
      const uint4 e = itab[i];
      const int a1 = (e.z >> 16) & 255, a2 = e.z >> 24, a3 = e.w & 255, a0 = N - (int)(e.w >> 8);
      const real* y = Dn + c * NQ;
      real v = real(a1) * y[e.y & 0xFFFF] + real(a2) * y[e.y >> 16] + real(a3) * y[e.z & 0xFFFF];
      if (a0 > 0) v += real(a0) * y[i];
      Rs[c * NP + i] = v / real(N);
    }
    // fluxes on the face coefficients
    for (int t = lane; t < 4 * NFP; t += 64) {
      const int f = t / NFP, m = t - f * NFP;
      const int po = fpos[f * NFP + m];
      const int cn = a.conn[4 * k + f];
      real jv[3], js[6];
      const real* gf = geo + 9 + 4 * f;
      const real nx = gf[1], ny = gf[2], nz = gf[3];
      if (cn >= 0) {
        const int64_t k2 = cn >> 2;
        const int pn = fpos[(cn & 3) * NFP + m];
#pragma unroll
        for (int c = 0; c < 3; ++c) jv[c] = a.q[((size_t)c * K + k2) * NP + pn] - Qs[c * NP + po];
#pragma unroll
        for (int c = 0; c < 6; ++c) js[c] = a.q[((size_t)(3 + c) * K + k2) * NP + pn] - Qs[(3 + c) * NP + po];
      } else if (a.wall == 0) {  // traction-free: sigma+ = -sigma, v+ = v
#pragma unroll
        for (int c = 0; c < 3; ++c) jv[c] = real(0);
#pragma unroll
        for (int c = 0; c < 6; ++c) js[c] = real(-2) * Qs[(3 + c) * NP + po];
      } else {  // rigid: v+ = -v, sigma+ = sigma
#pragma unroll
        for (int c = 0; c < 3; ++c) jv[c] = real(-2) * Qs[c * NP + po];
#pragma unroll
        for (int c = 0; c < 6; ++c) js[c] = real(0);
      }
      // A_n^T s = (sxx nx + sxy ny + sxz nz, sxy nx + syy ny + syz nz, sxz nx + syz ny + szz nz)
      auto AnT = [&](const real* s, real* o) {
        o[0] = s[0] * nx + s[5] * ny + s[4] * nz;
        o[1] = s[5] * nx + s[1] * ny + s[3] * nz;
        o[2] = s[4] * nx + s[3] * ny + s[2] * nz;
      };
      // A_n w = (nx w1, ny w2, nz w3, nz w2 + ny w3, nz w1 + nx w3, ny w1 + nx w2)
      auto An = [&](const real* w, real* o) {
        o[0] = nx * w[0];
        o[1] = ny * w[1];
        o[2] = nz * w[2];
        o[3] = nz * w[1] + ny * w[2];
        o[4] = nz * w[0] + nx * w[2];
        o[5] = ny * w[0] + nx * w[1];
      };
      real ats[3], anv[6], atanv[3], anats[6];
      AnT(js, ats);
      An(jv, anv);
      AnT(anv, atanv);
      An(ats, anats);
      real* Ff = Fs + f * 9 * NFP;
#pragma unroll
      for (int c = 0; c < 3; ++c) Ff[c * NFP + m] = real(0.5) * ats[c] + real(0.5) * a.tau_v * atanv[c];
#pragma unroll
      for (int c = 0; c < 6; ++c) Ff[(3 + c) * NFP + m] = real(0.5) * anv[c] + real(0.5) * a.tau_s * anats[c];
    }
    wsync();
    // lift: r[c][i] += sum_f Fscale_f sum_m L^f[i][m] F[f][c][m]
    for (int t = lane; t < 9 * NP; t += 64) {
      const int c = t / NP, i = t - c * NP;
      real r = Rs[c * NP + i];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const real sc = geo[9 + 4 * f];
        const real* Lf = a.lift + ((size_t)f * NP + i) * NFP;
        const real* Ff = Fs + (f * 9 + c) * NFP;
        real s = real(0);
        for (int m = 0; m < NFP; ++m) s += Lf[m] * Ff[m];
        r += sc * s;
      }
      a.out[((size_t)c * K + k) * NP + i] = r;
    }
    wsync();  // the slice is reused by the next element
  }
}

template <typename real, int N>
int launch_typed(const ElasticRhsArgs<real>& a, void* stream) {
  constexpr int WPB = ElRhsLayout<real, N>::WAVES;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t want = (a.K + WPB - 1) / WPB;
  const int64_t cap = (int64_t)(ncu > 0 ? ncu : 256) * 16;
  const int64_t blocks = want < cap ? want : cap;
  hipLaunchKernelGGL((elastic_rhs_kernel<real, N>), dim3((unsigned)blocks), dim3(64 * WPB), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace

template <typename real>
int launch_elastic_rhs(int N, const ElasticRhsArgs<real>& a, void* stream) {
  if (a.K <= 0) return 0;
  switch (N) {
    case 1: return launch_typed<real, 1>(a, stream);
    case 2: return launch_typed<real, 2>(a, stream);
    case 3: return launch_typed<real, 3>(a, stream);
    case 4: return launch_typed<real, 4>(a, stream);
    case 5: return launch_typed<real, 5>(a, stream);
    case 6: return launch_typed<real, 6>(a, stream);
    case 7: return launch_typed<real, 7>(a, stream);
    case 8: return launch_typed<real, 8>(a, stream);
    case 9: return launch_typed<real, 9>(a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template int launch_elastic_rhs<double>(int, const ElasticRhsArgs<double>&, void*);
template int launch_elastic_rhs<float>(int, const ElasticRhsArgs<float>&, void*);

}  // namespace bbw
