// Weight-adjusted update of the elastic velocity-stress system (paper Section 2.2, eq. ewadg):
// with the DG right-hand side r = (r_v, r_sigma) before the weight adjustment, the update is
//   v'_i     = Pi_N(rho^{-1} r_v_i)                         i = 1, 2, 3
//   sigma'_i = Pi_N(lambda tr(r_sigma) + 2 mu r_sigma_i)     i = xx, yy, zz
//   sigma'_s = Pi_N(mu r_sigma_s)                            s = yz, xz, xy
// (isotropic C, Voigt order xx, yy, zz, yz, xz, xy), i.e. the matrix-weighted weight-adjusted
// inverse (I (x) M^{-1}) M_C (I (x) M^{-1}) applied as scalar Bernstein products of degree
// N + M (eq. mcoeff) followed by 9 scalar projections: M one-degree reductions to degree N
// and the telescoped projection sum_j c_j E^N_{N-j} (E^N_{N-j})^T (Theorem 5.1).
//
// One wavefront per element (grid-stride over elements), everything in its LDS slice.
// Coefficients are in the graded order of the library, pos(a1, a2, a3) =
// dimp(s-1) + a3 (2s + 3 - a3)/2 + a2 with s = a1 + a2 + a3, the same position at every
// degree >= s, so a lane keeps one multi-index per slot across all levels.
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

__device__ __forceinline__ int gpos(int a1, int a2, int a3) {
  const int s = a1 + a2 + a3;
  return dimp(s - 1) + a3 * (2 * s + 3 - a3) / 2 + a2;
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ constexpr double factd(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

template <int N, int M>
struct ElasticLayout {
  static constexpr int NP = dimp(N), NH = dimp(N + M), MP = dimp(M);
  static constexpr int SH = (NH + 63) / 64;  // item slots of the product degree
  static constexpr int LEV = [] {            // levels r_0 .. r_N of the telescoping
    int t = 0;
    for (int j = 0; j <= N; ++j) t += dimp(N - j);
    return t;
  }();
  // X: 9 inputs and the trace, scaled by 1/alpha!; H, T: product and reduction ping-pong
  static constexpr int OFF_X = 0, OFF_H = 10 * NP, OFF_T = OFF_H + NH, OFF_L = OFF_T + NH, TOTAL = OFF_L + LEV;
  static constexpr int PTAB = MP * NH;  // byte table pos(gamma - beta), 255 where it does not exist
  template <typename real>
  static constexpr int waves() {
    const int per = TOTAL * (int)sizeof(real);
    const int room = 61440 - PTAB;
    return room / per >= 4 ? 4 : (room / per >= 1 ? room / per : 1);
  }
};

__host__ __device__ constexpr int lev_base(int N, int j) {  // start of level j (degree N - j)
  int t = 0;
  for (int i = 0; i < j; ++i) t += dimp(N - i);
  return t;
}

template <typename real, int N, int M, int WPB>
__global__ __launch_bounds__(64 * WPB) void elastic_update_kernel(ElasticArgs<real> a) {
  using L = ElasticLayout<N, M>;
  constexpr int NP = L::NP, NH = L::NH, MP = L::MP, SH = L::SH;
  __shared__ real smem[WPB * L::TOTAL];
  __shared__ uint8_t ptab[L::PTAB];
  static_assert(dimp(N) < 255, "product positions must fit a byte");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  real* const X = smem + wave * L::TOTAL + L::OFF_X;
  real* const H = smem + wave * L::TOTAL + L::OFF_H;
  real* const T = smem + wave * L::TOTAL + L::OFF_T;
  real* const LV = smem + wave * L::TOTAL + L::OFF_L;

  // per-slot multi-index of item lane + 64 s (graded order), found once
  int m1[SH], m2[SH], m3[SH];
#pragma unroll
  for (int s = 0; s < SH; ++s) {
    const int item = lane + 64 * s;
    int d = 0;
    while (d < N + M && dimp(d) <= item) ++d;  // degree of the item
    int r = item - dimp(d - 1), a3 = 0;
    while (a3 < d && r >= d + 1 - a3) r -= d + 1 - a3, ++a3;
    m3[s] = a3;
    m2[s] = r;
    m1[s] = d - a3 - r;
  }
  // graded-order neighbours of each slot, with D(s) = (s+1)(s+2)/2, s = |a|:
  //   pos(a+e1) = pos + D(s) + a3, pos(a+e2) = pos(a+e1) + 1, pos(a+e3) = pos + D(s) + s + 2,
  //   pos(a-e1) = pos - D(s-1) - a3, pos(a-e2) = pos - D(s-1) - a3 - 1, pos(a-e3) = pos - D(s-1) - s - 1
  int up1[SH], up2[SH], up3[SH], dn1[SH], dn2[SH], dn3[SH];
#pragma unroll
  for (int s = 0; s < SH; ++s) {
    const int i = lane + 64 * s, sa = m1[s] + m2[s] + m3[s];
    const int du = (sa + 1) * (sa + 2) / 2, dd = sa * (sa + 1) / 2;
    up1[s] = i + du + m3[s];
    up2[s] = up1[s] + 1;
    up3[s] = i + du + sa + 2;
    dn1[s] = m1[s] > 0 ? i - dd - m3[s] : 0;
    dn2[s] = m2[s] > 0 ? i - dd - m3[s] - 1 : 0;
    dn3[s] = m3[s] > 0 ? i - dd - sa - 1 : 0;
  }
  // the product table, once per workgroup: ptab[b][i] = pos(gamma_i - beta_b) or 255
  for (int t = threadIdx.x; t < L::PTAB; t += 64 * WPB) {
    const int b = t / NH, i = t - (t / NH) * NH;
    int d = 0;
    while (d < N + M && dimp(d) <= i) ++d;
    int r = i - dimp(d - 1), g3 = 0;
    while (g3 < d && r >= d + 1 - g3) r -= d + 1 - g3, ++g3;
    const int g2 = r, g1 = d - g3 - r, g0 = N + M - d;
    int sb = 0;
    while (sb < M && dimp(sb) <= b) ++sb;
    int q = b - dimp(sb - 1), b3 = 0;
    while (b3 < sb && q >= sb + 1 - b3) q -= sb + 1 - b3, ++b3;
    const int b2 = q, b1 = sb - b3 - q, b0 = M - sb;
    const bool ok = g1 >= b1 && g2 >= b2 && g3 >= b3 && g0 >= b0;
    ptab[t] = ok ? (uint8_t)gpos(g1 - b1, g2 - b2, g3 - b3) : (uint8_t)255;
  }
  __syncthreads();
  // 1/alpha! of the item as a degree-N coefficient, and kappa gamma! as a degree-(N+M) one
  constexpr double kappa = factd(N) * factd(M) / factd(N + M);
  real invN[SH], facH[SH];
#pragma unroll
  for (int s = 0; s < SH; ++s) {
    const int sa = m1[s] + m2[s] + m3[s];
    const double af = factd(m1[s]) * factd(m2[s]) * factd(m3[s]);
    invN[s] = sa <= N ? real(1.0 / (factd(N - sa) * af)) : real(0);
    facH[s] = real(kappa * factd(N + M - sa) * af);
  }
  const int64_t stride = (int64_t)gridDim.x * WPB;
  for (int64_t k = (int64_t)blockIdx.x * WPB + wave; k < a.K; k += stride) {
    // inputs scaled by 1/alpha! (a0 = N - |a| included), and the trace of the normal stresses
#pragma unroll
    for (int s = 0; s < SH; ++s) {
      const int i = lane + 64 * s;
      if (s * 64 < NP && i < NP) {
        const real inv = invN[s];
        real tr = real(0);
        for (int f = 0; f < 9; ++f) {
          const real x = a.r[((size_t)f * a.K + k) * NP + i] * inv;
          X[f * NP + i] = x;
          if (f >= 3 && f < 6) tr += x;
        }
        X[9 * NP + i] = tr;
      }
    }
    const real* wr = a.rho_inv + (size_t)k * MP;
    const real* wl = a.lam + (size_t)k * MP;
    const real* wm = a.mu + (size_t)k * MP;
    wsync();
    for (int c = 0; c < 9; ++c) {
      // product h = w1 f1 (+ w2 f2) in degree N + M (eq. mcoeff, scaled form)
      const real* w1 = c < 3 ? wr : (c < 6 ? wl : wm);
      const int f1 = c < 3 ? c : (c < 6 ? 9 : c);
      const real s1 = real(1);
      const real* w2 = c >= 3 && c < 6 ? wm : nullptr;
      const int f2 = c;
      const real s2 = real(2);
#pragma unroll
      for (int s = 0; s < SH; ++s) {
        const int i = lane + 64 * s;
        if (i < NH) {
          real h = real(0);
          int b = 0;
#pragma unroll
          for (int sb = 0; sb <= M; ++sb)
#pragma unroll
            for (int b3 = 0; b3 <= sb; ++b3)
#pragma unroll
              for (int b2 = 0; b2 <= sb - b3; ++b2, ++b) {
                const int p = ptab[b * NH + i];
                if (p == 255) continue;
                const real bf = real(1.0 / (factd(M - sb) * factd(sb - b2 - b3) * factd(b2) * factd(b3)));
                h += X[f1 * NP + p] * (s1 * w1[b] * bf);
                if (w2) h += X[f2 * NP + p] * (s2 * w2[b] * bf);
              }
          H[i] = h * facH[s];
        }
      }
      wsync();
      // M one-degree reductions N+M -> N: y_a = [(a0+1) x_a + sum_j (a_j + 1) x_{a+e_j}] / n
      real* src = H;
      for (int n = N + M; n > N; --n) {
        real* dst = (n - 1 == N) ? LV : (src == H ? T : H);
        const int cnt = dimp(n - 1);
#pragma unroll
        for (int s = 0; s < SH; ++s) {
          const int i = lane + 64 * s;
          if (i < cnt) {
            const int a1 = m1[s], a2 = m2[s], a3 = m3[s], a0 = n - 1 - a1 - a2 - a3;
            dst[i] = (real(a0 + 1) * src[i] + real(a1 + 1) * src[up1[s]] + real(a2 + 1) * src[up2[s]] +
                      real(a3 + 1) * src[up3[s]]) / real(n);
          }
        }
        wsync();
        src = dst;
      }
      if constexpr (M == 0) {  // no reduction: level 0 is the product itself
#pragma unroll
        for (int s = 0; s < SH; ++s) {
          const int i = lane + 64 * s;
          if (i < NP) LV[i] = H[i];
        }
        wsync();
      }
      // downward sweep: level j = reduction of level j - 1 (degree N - j + 1 -> N - j)
      for (int j = 1; j <= N; ++j) {
        const int n = N - j + 1;
        const real* lsrc = LV + lev_base(N, j - 1);
        real* ldst = LV + lev_base(N, j);
        const int cnt = dimp(n - 1);
#pragma unroll
        for (int s = 0; s < SH; ++s) {
          const int i = lane + 64 * s;
          if (i < cnt) {
            const int a1 = m1[s], a2 = m2[s], a3 = m3[s], a0 = n - 1 - a1 - a2 - a3;
            ldst[i] = (real(a0 + 1) * lsrc[i] + real(a1 + 1) * lsrc[up1[s]] + real(a2 + 1) * lsrc[up2[s]] +
                       real(a3 + 1) * lsrc[up3[s]]) / real(n);
          }
        }
        wsync();
      }
      // upward sweep: s_N = c_N r_N; s_j = c_j r_j + E s_{j+1}, (E y)_g = sum_{g_j > 0} g_j / n y_{g - e_j}
      if (lane == 0) LV[lev_base(N, N)] *= a.cj[N];
      wsync();
      for (int j = N - 1; j >= 0; --j) {
        const int n = N - j;  // degree of level j
        real* lo = LV + lev_base(N, j);
        const real* hi = LV + lev_base(N, j + 1);
        const int cnt = dimp(n);
        const real cj = a.cj[j];
        real v[SH];
#pragma unroll
        for (int s = 0; s < SH; ++s) {
          const int i = lane + 64 * s;
          v[s] = real(0);
          if (i < cnt) {
            const int a1 = m1[s], a2 = m2[s], a3 = m3[s], a0 = n - a1 - a2 - a3;
            real e = real(0);
            if (a0 > 0) e += real(a0) * hi[i];
            e += real(a1) * hi[dn1[s]] + real(a2) * hi[dn2[s]] + real(a3) * hi[dn3[s]];  // zero weight where a_j = 0
            v[s] = cj * lo[i] + e / real(n);
          }
        }
        wsync();  // every lane has read level j before it is overwritten
#pragma unroll
        for (int s = 0; s < SH; ++s) {
          const int i = lane + 64 * s;
          if (i < cnt) lo[i] = v[s];
        }
        wsync();
      }
#pragma unroll
      for (int s = 0; s < SH; ++s) {
        const int i = lane + 64 * s;
        if (s * 64 < NP && i < NP) a.out[((size_t)c * a.K + k) * NP + i] = LV[i];
      }
      wsync();  // H, T and the levels are reused by the next component
    }
  }
}

template <typename real, int N, int M>
int launch_typed(const ElasticArgs<real>& a, void* stream) {
  constexpr int WPB = ElasticLayout<N, M>::template waves<real>();
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t want = (a.K + WPB - 1) / WPB;
  const int64_t cap = (int64_t)(ncu > 0 ? ncu : 256) * 16;
  const int64_t blocks = want < cap ? want : cap;
  hipLaunchKernelGGL((elastic_update_kernel<real, N, M, WPB>), dim3((unsigned)blocks), dim3(64 * WPB), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

template <typename real, int N>
int launch_n(int M, const ElasticArgs<real>& a, void* stream) {
  switch (M) {
    case 0: return launch_typed<real, N, 0>(a, stream);
    case 1: if constexpr (N >= 1) return launch_typed<real, N, 1>(a, stream); break;
    case 2: if constexpr (N >= 2) return launch_typed<real, N, 2>(a, stream); break;
    case 3: if constexpr (N >= 3) return launch_typed<real, N, 3>(a, stream); break;
    case 4: if constexpr (N >= 4) return launch_typed<real, N, 4>(a, stream); break;
    default: break;
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace

template <typename real>
int launch_elastic_update(int N, int M, const ElasticArgs<real>& a, void* stream) {
  if (a.K <= 0) return 0;
  switch (N) {
    case 1: return launch_n<real, 1>(M, a, stream);
    case 2: return launch_n<real, 2>(M, a, stream);
    case 3: return launch_n<real, 3>(M, a, stream);
    case 4: return launch_n<real, 4>(M, a, stream);
    case 5: return launch_n<real, 5>(M, a, stream);
    case 6: return launch_n<real, 6>(M, a, stream);
    case 7: return launch_n<real, 7>(M, a, stream);
    case 8: return launch_n<real, 8>(M, a, stream);
    case 9: return launch_n<real, 9>(M, a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template int launch_elastic_update<double>(int, int, const ElasticArgs<double>&, void*);
template int launch_elastic_update<float>(int, int, const ElasticArgs<float>&, void*);

}  // namespace bbw
