// Weight-adjusted update of the elastic velocity-stress system (paper Section 3.2, eq. ewadg):
// with the DG right-hand side r = (r_v, r_sigma) before the weight adjustment, the update is
//   v'_i     = Pi_N(rho^{-1} r_v_i)                         i = 1, 2, 3
//   sigma'_i = Pi_N(lambda tr(r_sigma) + 2 mu r_sigma_i)     i = xx, yy, zz
//   sigma'_s = Pi_N(mu r_sigma_s)                            s = yz, xz, xy
// (isotropic C, Voigt order xx, yy, zz, yz, xz, xy), i.e. the matrix-weighted weight-adjusted
// inverse (I (x) M^{-1}) M_C (I (x) M^{-1}) applied as scalar Bernstein products of degree
// N + M (eq. mcoeff) followed by 9 scalar projections: M one-degree reductions to degree N
// and the telescoped projection sum_j c_j E^N_{N-j} (E^N_{N-j})^T (Theorem 5.3).
//
// One wavefront per element (grid-stride over elements), everything in its LDS slice; the 9
// components go through the projection in groups (see ElasticLayout).
// Coefficients are in the graded order of the library, pos(a1, a2, a3) =
// dimp(s-1) + a3 (2s + 3 - a3)/2 + a2 with s = a1 + a2 + a3, the same position at every
// degree >= s, so a lane keeps one multi-index per slot across all levels.
#include <type_traits>

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

__host__ __device__ constexpr int lev_base(int N, int j) {  // start of level j (degree N - j)
  int t = 0;
  for (int i = 0; i < j; ++i) t += dimp(N - i);
  return t;
}

// Components are processed in groups of G (up to N = 4 9, 3 or 1, the largest whose buffers
// fit; from N = 5 always 1): every phase of the projection runs over G x (coefficients) items
// at once, so a wavefront syncs (1 + M + 2N) times per group instead of per component and the
// small levels fill more lanes.
template <typename real, int N, int M>
constexpr int elastic_tables() {  // product positions (bytes), stencil table (16 B), gamma! kappa
  return dimp(M) * dimp(N + M) + 16 * dimp(N + M) + (int)sizeof(real) * dimp(N + M);
}
// NC = 9: the elastic update (9 inputs and the trace, 3 media); NC = 1: one field and one
// weight (the acoustic update Pi_N(c^2_M r)).
// FP32 projections of degree N >= BBW_TELE64_MIN_N run the telescoping in FP64 (the levels
// as doubles): the alternating c_j amplify the rounding of float sweeps.
template <typename real, int N, int M>
constexpr bool elastic_tele64() {
  return sizeof(real) == 4 && N >= BBW_TELE64_MIN_N && M > 0;
}
template <typename real, int N, int M, int NC>
constexpr int elastic_per_wave(int G) {
  constexpr int XF = NC == 9 ? 10 : 1, NW = NC == 9 ? 3 : 1;
  constexpr int LV = (elastic_tele64<real, N, M>() ? 2 : 1) * lev_base(N, N + 1);
  return (XF * dimp(N) + NW * dimp(M) + G * (dimp(N + M) + dimp(N + M - 1) + LV) + 2) * (int)sizeof(real);
}

// LDS bytes a wavefront's buffers may take when choosing the group size (occupancy against
// fewer, wider phases).
#ifndef BBW_EL_WAVE_BYTES
#define BBW_EL_WAVE_BYTES 8192
#endif

template <typename real, int N, int M, int NC>
constexpr int elastic_group() {
  constexpr int T = elastic_tables<real, N, M>();
  auto fits = [](int G) {
    const int w = elastic_per_wave<real, N, M, NC>(G);
    return w <= BBW_EL_WAVE_BYTES && w + T <= 61440;
  };
  // From N = 5 one component per group, whose table entries sit in registers (below), beats
  // wider groups whatever the LDS allows: FP32 N = 5, M = 1..3 took 0.77 / 1.23 / 2.45 ms
  // against 0.86 / 1.62 / 3.41 with groups of 3 (196,608 tets); up to N = 4 the groups win
  // (N = 2, M = 1: 0.21 ms against 0.50 in FP64).
  return NC == 1 || N >= 5 ? 1 : (fits(9) ? 9 : (fits(3) ? 3 : 1));
}
template <typename real, int N, int M, int NC>
constexpr int elastic_waves() {
  constexpr int room =
      (61440 - elastic_tables<real, N, M>()) / elastic_per_wave<real, N, M, NC>(elastic_group<real, N, M, NC>());
  return room >= 4 ? 4 : (room >= 1 ? room : 1);
}

// One-component groups hold their per-position table entries in registers up to this many
// 64-position slots of the product degree (BBW_EL_REG_SLOTS forces a limit). Measured at
// 196,608 tets against reading them from LDS in every phase: 1.1-1.55x faster for the 9-field
// update and 1.2-1.8x for the one-field update from N = 5; FP64 N = 9, M = 4 (9 slots) was
// 4% slower, so FP64 stops at 8 slots.
#ifndef BBW_EL_REG_SLOTS
#define BBW_EL_REG_SLOTS -1
#endif
constexpr int el_reg_slots(int bytes) { return BBW_EL_REG_SLOTS >= 0 ? BBW_EL_REG_SLOTS : (bytes == 8 ? 8 : 16); }

template <typename real, int N, int M, int NC>
struct ElasticLayout {
  static constexpr int NP = dimp(N), NH = dimp(N + M), MP = dimp(M), NB = dimp(N + M - 1);
  static constexpr int LEV = lev_base(N, N + 1);  // levels r_0 .. r_N
  static constexpr int XF = NC == 9 ? 10 : 1, NW = NC == 9 ? 3 : 1;
  static constexpr int G = elastic_group<real, N, M, NC>(), WAVES = elastic_waves<real, N, M, NC>();
  static constexpr bool TELE64 = elastic_tele64<real, N, M>();
  // the levels start 8-byte aligned (doubles with TELE64), and so does every wave's slice
  static constexpr int OFF_X = 0, OFF_W = XF * NP, OFF_A = OFF_W + NW * MP, OFF_B = OFF_A + G * NH,
                       OFF_L = (OFF_B + G * NB + 1) / 2 * 2, TOTAL = (OFF_L + (TELE64 ? 2 : 1) * G * LEV + 1) / 2 * 2;
};

template <typename real, int N, int M, int NC>
__global__ __launch_bounds__((64 * ElasticLayout<real, N, M, NC>::WAVES)) void weighted_projection_kernel(ElasticArgs<real> a) {
  using L = ElasticLayout<real, N, M, NC>;
  constexpr int NP = L::NP, NH = L::NH, MP = L::MP, NB = L::NB, LEV = L::LEV, G = L::G, WPB = L::WAVES;
  static_assert(NP < 255, "product positions must fit a byte");
  __shared__ __attribute__((aligned(16))) real smem[WPB * L::TOTAL];
  __shared__ uint8_t ptab[MP * NH];
  __shared__ uint4 itab[NH];
  __shared__ real facH[NH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  real* const X = smem + wave * L::TOTAL + L::OFF_X;
  real* const Wt = smem + wave * L::TOTAL + L::OFF_W;
  real* const A = smem + wave * L::TOTAL + L::OFF_A;
  real* const B = smem + wave * L::TOTAL + L::OFF_B;
  real* const LV = smem + wave * L::TOTAL + L::OFF_L;
  double* const LVD = reinterpret_cast<double*>(smem + wave * L::TOTAL + L::OFF_L);  // the levels (L::TELE64)

  // ---- per-block tables -------------------------------------------------------------
  // itab[i] for the multi-index a at graded position i (s = |a|, D(s) = (s+1)(s+2)/2):
  //   x: pos(a+e1) = i + D(s) + a3 | pos(a+e3) = i + D(s) + s + 2 << 16  (pos(a+e2) = pos(a+e1) + 1)
  //   y: pos(a-e1) = i - D(s-1) - a3 | pos(a-e2) = i - D(s-1) - a3 - 1 << 16 (0 where a_j = 0)
  //   z: pos(a-e3) = i - D(s-1) - s - 1 (0 where a3 = 0) | a1 << 16 | a2 << 24;  w: a3 | s << 8
  constexpr double kappa = factd(N) * factd(M) / factd(N + M);
  for (int i = threadIdx.x; i < NH; i += 64 * WPB) {
    int d = 0;
    while (d < N + M && dimp(d) <= i) ++d;
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
    facH[i] = real(kappa * factd(N + M - d) * factd(a1) * factd(a2) * factd(a3));
  }
  for (int t = threadIdx.x; t < MP * NH; t += 64 * WPB) {  // ptab[b][i] = pos(gamma_i - beta_b) or 255
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

  // With one component per group, item i of every phase is position i itself, so a lane
  // visits the same positions lane + 64 s in every phase and element: their table entries
  // and factors are read once into registers, and a phase issues only its value reads.
  constexpr int S = (NH + 63) / 64;
  constexpr bool REG = G == 1 && S <= el_reg_slots((int)sizeof(real));
  uint4 es[REG ? S : 1];
  real fh[REG ? S : 1];
  if constexpr (REG) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = lane + 64 * s;
      es[s] = i < NH ? itab[i] : uint4{0, 0, 0, 0};
      fh[s] = i < NH ? facH[i] : real(0);
    }
  }
  // 1/alpha! (a0 = N - |a| included) for the inputs, 1/beta! for the media
  constexpr int SN = (NP + 63) / 64, SW = (L::NW * MP + 63) / 64;
  real xinv[SN], winv[SW];
#pragma unroll
  for (int s = 0; s < SN; ++s) {
    const int i = lane + 64 * s < NP ? lane + 64 * s : 0;
    const uint4 e = itab[i];
    const int a1 = (e.z >> 16) & 255, a2 = e.z >> 24, a3 = e.w & 255, sa = e.w >> 8;
    xinv[s] = real(1.0 / (factd(N - sa) * factd(a1) * factd(a2) * factd(a3)));
  }
#pragma unroll
  for (int s = 0; s < SW; ++s) {
    const int t = lane + 64 * s < L::NW * MP ? lane + 64 * s : 0;
    const uint4 e = itab[t - (t / MP) * MP];  // beta at position b (|beta| <= M)
    const int b1 = (e.z >> 16) & 255, b2 = e.z >> 24, b3 = e.w & 255, sb = e.w >> 8;
    winv[s] = real(1.0 / (factd(M - sb) * factd(b1) * factd(b2) * factd(b3)));
  }

  // visits items (component cl of the group, position i < cnt) with the entry of i
  auto items = [&](int cnt, auto&& f) {
    if constexpr (REG) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int i = lane + 64 * s;
        if (64 * s < cnt && i < cnt) f(0, i, s, es[s]);
      }
    } else {
      for (int t = lane; t < G * cnt; t += 64) {
        const int cl = t / cnt, i = t - cl * cnt;
        f(cl, i, 0, itab[i]);
      }
    }
  };

  // one reduction (E^n_{n-1})^T over G components: y_a = [(a0+1) x_a + sum_j (a_j+1) x_{a+e_j}] / n,
  // in the source's precision (stored in the destination's)
  auto reduce = [&](const auto* src, int sst, auto* dst, int dstr, int n) {
    using T = std::remove_cv_t<std::remove_pointer_t<decltype(src)>>;
    const T inv = T(1) / T(n);
    items(dimp(n - 1), [&](int cl, int i, int, const uint4 e) {
      const int a1 = (e.z >> 16) & 255, a2 = e.z >> 24, a3 = e.w & 255, a0 = n - 1 - (int)(e.w >> 8);
      const T* x = src + cl * sst;
      const int u1 = e.x & 0xFFFF, u3 = e.x >> 16;
      dst[cl * dstr + i] = inv * (T(a0 + 1) * x[i] + T(a1 + 1) * x[u1] + T(a2 + 1) * x[u1 + 1] + T(a3 + 1) * x[u3]);
    });
    wsync();
  };

  const int64_t stride = (int64_t)gridDim.x * WPB;
  for (int64_t k = (int64_t)blockIdx.x * WPB + wave; k < a.K; k += stride) {
    // inputs scaled by 1/alpha! (a0 = N - |a| included), the trace of the normal stresses, and
    // the media scaled by 1/beta!
#pragma unroll
    for (int s = 0; s < SN; ++s) {
      const int i = lane + 64 * s;
      if (i < NP) {
        real tr = real(0);
#pragma unroll
        for (int f = 0; f < NC; ++f) {
          const real x = a.r[((size_t)f * a.K + k) * NP + i] * xinv[s];
          X[f * NP + i] = x;
          if (f >= 3 && f < 6) tr += x;
        }
        if constexpr (NC == 9) X[9 * NP + i] = tr;
      }
    }
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      const int t = lane + 64 * s;
      if (t < L::NW * MP) {
        const int w = t / MP, b = t - w * MP;
        const real* src = w == 0 ? a.rho_inv : (w == 1 ? a.lam : a.mu);
        Wt[t] = src[(size_t)k * MP + b] * winv[s];
      }
    }
    wsync();
    for (int c0 = 0; c0 < NC; c0 += G) {
      // products (eq. mcoeff, scaled form): velocities rho^{-1} v_i, normal stresses
      // lambda tr + 2 mu sigma_i, shear stresses mu sigma_s
      real* const P = M > 0 ? A : LV;  // with M = 0 the product is level 0 itself
      const int pst = M > 0 ? NH : LEV;
      items(NH, [&](int cl, int i, int sl, const uint4) {
        const int c = c0 + cl;
        const int f1 = NC == 1 ? 0 : (c < 3 ? c : (c < 6 ? 9 : c));
        const real* w1 = Wt + (NC == 1 ? 0 : (c < 3 ? 0 : (c < 6 ? 1 : 2))) * MP;
        const bool two = NC == 9 && c >= 3 && c < 6;
        real h = real(0);
#pragma unroll
        for (int b = 0; b < MP; ++b) {
          const int p = ptab[b * NH + i];
          if (p == 255) continue;
          h += X[f1 * NP + p] * w1[b];
          if (two) h += real(2) * X[c * NP + p] * Wt[2 * MP + b];
        }
        P[cl * pst + i] = h * (REG ? fh[sl] : facH[i]);
      });
      wsync();
      // M reductions N+M -> N (ping-pong A <-> B, the last into level 0)
      if constexpr (M > 0) {
        const real* src = A;
        int sst = NH;
#pragma unroll
        for (int n = N + M; n > N; --n) {
          const bool last = n - 1 == N;
          if (L::TELE64 && last) {
            reduce(src, sst, LVD, LEV, n);  // level 0, widened
            break;
          }
          real* dst = last ? LV : (src == A ? B : A);
          const int dstr = last ? LEV : (src == A ? NB : NH);
          reduce(src, sst, dst, dstr, n);
          src = dst;
          sst = dstr;
        }
      }
      if constexpr (L::TELE64) {
        // FP64 telescoping (FP32 state): the sweeps below on doubles, the result rounded to
        // float into A (free once the reductions are done), where the writes read it
#pragma unroll
        for (int j = 1; j <= N; ++j) reduce(LVD + lev_base(N, j - 1), LEV, LVD + lev_base(N, j), LEV, N - j + 1);
        if (lane < G) LVD[lane * LEV + lev_base(N, N)] *= a.cjd[N];
        wsync();
#pragma unroll
        for (int j = N - 1; j >= 0; --j) {
          const int n = N - j;
          const double cj = a.cjd[j], inv = 1.0 / double(n);
          items(dimp(n), [&](int cl, int i, int, const uint4 e) {
            const int a1 = (e.z >> 16) & 255, a2 = e.z >> 24, a3 = e.w & 255, a0 = n - (int)(e.w >> 8);
            double* lo = LVD + cl * LEV + lev_base(N, j);
            const double* hi = LVD + cl * LEV + lev_base(N, j + 1);
            double el = double(a1) * hi[e.y & 0xFFFF] + double(a2) * hi[e.y >> 16] + double(a3) * hi[e.z & 0xFFFF];
            if (a0 > 0) el += double(a0) * hi[i];
            lo[i] = cj * lo[i] + inv * el;  // only this item reads lo[i]
          });
          wsync();
        }
        for (int t = lane; t < G * NP; t += 64) {
          const int cl = t / NP, i = t - cl * NP;
          A[cl * NP + i] = real(LVD[cl * LEV + i]);
        }
        wsync();
      } else {
        // downward sweep: level j = reduction of level j - 1
#pragma unroll
        for (int j = 1; j <= N; ++j) reduce(LV + lev_base(N, j - 1), LEV, LV + lev_base(N, j), LEV, N - j + 1);
        // upward sweep: s_N = c_N r_N; s_j = c_j r_j + E s_{j+1}, (E y)_g = sum_{g_j > 0} g_j / n y_{g - e_j}
        if (lane < G) LV[lane * LEV + lev_base(N, N)] *= a.cj[N];
        wsync();
#pragma unroll
        for (int j = N - 1; j >= 0; --j) {
          const int n = N - j;
          const real cj = a.cj[j], inv = real(1) / real(n);
          items(dimp(n), [&](int cl, int i, int, const uint4 e) {
            const int a1 = (e.z >> 16) & 255, a2 = e.z >> 24, a3 = e.w & 255, a0 = n - (int)(e.w >> 8);
            real* lo = LV + cl * LEV + lev_base(N, j);
            const real* hi = LV + cl * LEV + lev_base(N, j + 1);
            real el = real(a1) * hi[e.y & 0xFFFF] + real(a2) * hi[e.y >> 16] + real(a3) * hi[e.z & 0xFFFF];
            if (a0 > 0) el += real(a0) * hi[i];
            lo[i] = cj * lo[i] + inv * el;  // only this item reads lo[i]
          });
          wsync();
        }
      }
      const real* RES = L::TELE64 ? A : LV;  // the projected group
      constexpr int RST = L::TELE64 ? NP : LEV;
      if (a.res) {  // a low-storage RK stage (uniform branch); res and q never alias
        real* __restrict__ rs = a.res;
        real* __restrict__ qs = a.q;
#pragma unroll 4
        for (int t = lane; t < G * NP; t += 64) {
          const int cl = t / NP, i = t - cl * NP;
          const size_t idx = ((size_t)(c0 + cl) * a.K + k) * NP + i;
          const real r2 = a.rk_a * rs[idx] + a.dt * RES[cl * RST + i];
          rs[idx] = r2;
          qs[idx] += a.rk_b * r2;
        }
      } else {
        for (int t = lane; t < G * NP; t += 64) {
          const int cl = t / NP, i = t - cl * NP;
          a.out[((size_t)(c0 + cl) * a.K + k) * NP + i] = RES[cl * RST + i];
        }
      }
      wsync();  // the buffers are reused by the next group and element
    }
  }
}

template <typename real, int N, int M, int NC>
int launch_typed(const ElasticArgs<real>& a, void* stream) {
  constexpr int WPB = ElasticLayout<real, N, M, NC>::WAVES;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t want = (a.K + WPB - 1) / WPB;
  const int64_t cap = (int64_t)(ncu > 0 ? ncu : 256) * 16;
  const int64_t blocks = want < cap ? want : cap;
  hipLaunchKernelGGL((weighted_projection_kernel<real, N, M, NC>), dim3((unsigned)blocks), dim3(64 * WPB), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

template <typename real, int N, int NC>
int launch_n(int M, const ElasticArgs<real>& a, void* stream) {
  switch (M) {
    case 0: return launch_typed<real, N, 0, NC>(a, stream);
    case 1: if constexpr (N >= 1) return launch_typed<real, N, 1, NC>(a, stream); break;
    case 2: if constexpr (N >= 2) return launch_typed<real, N, 2, NC>(a, stream); break;
    case 3: if constexpr (N >= 3) return launch_typed<real, N, 3, NC>(a, stream); break;
    case 4: if constexpr (N >= 4) return launch_typed<real, N, 4, NC>(a, stream); break;
    default: break;
  }
  return (int)hipErrorInvalidValue;
}

template <typename real, int NC>
int launch_nc(int N, int M, const ElasticArgs<real>& a, void* stream) {
  if (a.K <= 0) return 0;
  switch (N) {
    case 1: return launch_n<real, 1, NC>(M, a, stream);
    case 2: return launch_n<real, 2, NC>(M, a, stream);
    case 3: return launch_n<real, 3, NC>(M, a, stream);
    case 4: return launch_n<real, 4, NC>(M, a, stream);
    case 5: return launch_n<real, 5, NC>(M, a, stream);
    case 6: return launch_n<real, 6, NC>(M, a, stream);
    case 7: return launch_n<real, 7, NC>(M, a, stream);
    case 8: return launch_n<real, 8, NC>(M, a, stream);
    case 9: return launch_n<real, 9, NC>(M, a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

template <typename real>
int launch_elastic_update(int N, int M, const ElasticArgs<real>& a, void* stream) {
  return launch_nc<real, 9>(N, M, a, stream);
}

template <typename real>
int launch_wadg_update(int N, int M, const ElasticArgs<real>& a, void* stream) {
  return launch_nc<real, 1>(N, M, a, stream);
}

template int launch_elastic_update<double>(int, int, const ElasticArgs<double>&, void*);
template int launch_elastic_update<float>(int, int, const ElasticArgs<float>&, void*);
template int launch_wadg_update<double>(int, int, const ElasticArgs<double>&, void*);
template int launch_wadg_update<float>(int, int, const ElasticArgs<float>&, void*);

}  // namespace bbw
