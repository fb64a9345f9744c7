// DG right-hand side of the elastic velocity-stress system before the weight adjustment
// (paper Section 3.2, the semi-discrete form after eq. ewave), isotropic or not (the media
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
//  * lift: L^f = E_L L_0 (Section 4): L_0 = (2N+3)/2 I + N^2/2 E E^T on the face flux, then a
//    chain of 2D degree reductions E^T, level i scaled by l_i = (-1)^i C(N, i)/(i + 1), and the
//    coefficient alpha takes level alpha_f at its face multi-index. One face at a time, so the
//    flux, the chain and its first reduction share one LDS region.
#include "bbwadg_internal.hpp"

namespace bbw {
namespace {

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Degree s = b1 + b2 of face position m in the graded order, m = s (s + 1) / 2 + b2, from a
// square root: floor((sqrt(8 m + 1.5) - 1) / 2) is s with a margin of at least 0.006 on
// either side for m < 64 (the 0.5 added under the root keeps the triangular numbers, where
// 8 m + 1 is a perfect square, clear of the rounding of v_sqrt_f32). A few VALU instructions
// instead of an LDS table read before the values a lift phase needs. The empty asm keeps
// the decode where it is used: hoisted out of the face loop, the decodes of every level
// would stay live in registers across it. Used from N = 6 (196,608 tets, ms per right-hand
// side, table / decode: FP64 N = 9 17.3 / 11.9, N = 6..8 and FP32 N = 6..9 within 1.2%
// either way); up to N = 5 the table read measured 1.5-6% faster and is kept there.
__device__ __forceinline__ int face_degree(int m) {
  asm volatile("" : "+v"(m));
  return (int)((__builtin_amdgcn_sqrtf(8.0f * (float)m + 1.5f) - 1.0f) * 0.5f);
}

// l_i = (-1)^i C(N, i) / (i + 1): factor of lift level i.
__host__ __device__ constexpr double lift_level(int N, int i) {
  double c = 1.0;
  for (int j = 1; j <= i; ++j) c = c * (N - i + j) / j;
  return (i % 2 ? -c : c) / (i + 1);
}

template <typename real, int N>
struct ElRhsLayout {
  static constexpr int NP = dimp(N), NQ = dimp(N - 1), NFP = dim2(N);
  // per wave: Qs [9][NP], the result Rs [9][NP] (unless REG), then a region used first for
  // the degree N-1 derivatives [9][NQ], then per face for the flux F [9][NFP] and the lift
  // chain [9][NP] (level i of degree N - i at offset sum_{i' < i} dim2(N - i')). With REG the result accumulates in registers instead (item
  // t = lane + 64 j of the [9][NP] output in slot j): that frees LDS where LDS limits the
  // wavefronts per CU (FP64 from N = 5, FP32 from N = 6; below, the registers cost more
  // occupancy than the LDS does, as measured on MI355X).
  static constexpr bool REG = sizeof(real) == 8 ? N >= 5 : N >= 6;
  static constexpr int OFF_Q = 0, OFF_R = 9 * NP, OFF_W = REG ? 9 * NP : 18 * NP, RJ = (9 * NP + 63) / 64;
  static constexpr int WSZ = 9 * NQ > 9 * (NFP + NP) ? 9 * NQ : 9 * (NFP + NP);
  static constexpr int TOTAL = OFF_W + WSZ;
  static constexpr bool DECODE = N >= 6;  // face positions decoded (face_degree), else a table
  static constexpr int TABLES = 16 * NP + 4 * NP + 4 * 4 * NFP + (DECODE ? 0 : 4 * NFP);
  static constexpr int per = TOTAL * (int)sizeof(real);
  static constexpr int WAVES = (61440 - TABLES) / per >= 4 ? 4 : ((61440 - TABLES) / per >= 1 ? (61440 - TABLES) / per : 1);
};

template <typename real, int N>
__global__ __launch_bounds__((64 * ElRhsLayout<real, N>::WAVES)) void elastic_rhs_kernel(ElasticRhsArgs<real> a) {
  using L = ElRhsLayout<real, N>;
  constexpr int NP = L::NP, NQ = L::NQ, NFP = L::NFP, WPB = L::WAVES;
  __shared__ real smem[WPB * L::TOTAL];
  __shared__ uint4 itab[NP];
  __shared__ uint32_t lpos[NP];  // byte f: chain position of coefficient i for face f
  __shared__ int fpos[4 * NFP];
  __shared__ int ftab[L::DECODE ? 1 : NFP];  // face position m at any degree: s | b2 << 8
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  real* const Qs = smem + wave * L::TOTAL + L::OFF_Q;
  real* const Rs = smem + wave * L::TOTAL + L::OFF_R;  // used only without REG
  real* const Dn = smem + wave * L::TOTAL + L::OFF_W;
  real* const Fs = Dn;                 // [9][NFP]
  real* const Cs = Dn + 9 * NFP;       // [9][NP]

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
    // lift gather: face f's vertices in ascending order without f, (b0, b1, b2) of alpha on
    // them; level j = alpha_f of degree N - j starts at sum_{i' < j} dim2(N - i')
    const int al[4] = {N - d, a1, a2, a3};
    uint32_t lp = 0;
    for (int f = 0; f < 4; ++f) {
      int vs[3], n = 0;
      for (int v = 0; v < 4; ++v)
        if (v != f) vs[n++] = v;
      const int j = al[f], b1 = al[vs[1]], b2 = al[vs[2]], sb = b1 + b2;
      int off = 0;
      for (int q = 0; q < j; ++q) off += dim2(N - q);
      lp |= (uint32_t)(off + sb * (sb + 1) / 2 + b2) << (8 * f);
    }
    lpos[i] = lp;
  }
  for (int i = threadIdx.x; i < 4 * NFP; i += 64 * WPB) fpos[i] = a.fpos[i];
  if constexpr (!L::DECODE) {
    for (int m = threadIdx.x; m < NFP; m += 64 * WPB) {
      int sb = 0;
      while ((sb + 1) * (sb + 2) / 2 <= m) ++sb;
      ftab[m] = sb | ((m - sb * (sb + 1) / 2) << 8);
    }
  }
  // degree sb and b2 of face position b (b1 = sb - b2)
  auto face_sb = [&](int b, int& sb, int& b2) {
    if constexpr (L::DECODE) {
      sb = face_degree(b);
      b2 = b - sb * (sb + 1) / 2;
    } else {
      sb = ftab[b] & 255;
      b2 = ftab[b] >> 8;
    }
  };
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
    real racc[L::REG ? L::RJ : 1];
    constexpr int UNR = L::REG ? L::RJ : 1;  // the LDS variant keeps rolled loops (fewer registers)
#pragma unroll UNR
    for (int j = 0; j < L::RJ; ++j) {
      const int t = lane + 64 * j;
      if constexpr (L::REG) racc[j] = real(0);
      if (t < 9 * NP) {
        const int c = t / NP, i = t - c * NP;
        const uint4 e = itab[i];
        const int a1 = (e.z >> 16) & 255, a2 = e.z >> 24, a3 = e.w & 255, a0 = N - (int)(e.w >> 8);
        const real* y = Dn + c * NQ;
        real v = real(a1) * y[e.y & 0xFFFF] + real(a2) * y[e.y >> 16] + real(a3) * y[e.z & 0xFFFF];
        if (a0 > 0) v += real(a0) * y[i];
        if constexpr (L::REG) racc[j] = v / real(N);
        else Rs[t] = v / real(N);  // t = c NP + i
      }
    }
    wsync();  // Dn is dead: its region holds the face work from here
    for (int f = 0; f < 4; ++f) {
      // flux on face f's coefficients
      const int cn = a.conn[4 * k + f];
      const real* gf = geo + 9 + 4 * f;
      const real nx = gf[1], ny = gf[2], nz = gf[3];
      for (int m = lane; m < NFP; m += 64) {
        const int po = fpos[f * NFP + m];
        // FP64 from N = 5: the neighbour's coefficients are loaded on every face (a wall face
        // loads its own element's as a stand-in and discards them), since loads under a branch
        // make the compiler wait for every outstanding load where the branch joins (N = 5:
        // 2.33 -> 1.85 ms per call at 196,608 tets). Elsewhere the branch form is kept: the
        // extra live values cost FP32 N = 7 a wave per SIMD (2.93 -> 3.83 ms).
        constexpr bool NB_ALWAYS = sizeof(real) == 8 && N >= 5;
        real jv[3], js[6];
        if constexpr (NB_ALWAYS) {
          const bool inner = cn >= 0;
          const int64_t k2 = inner ? (int64_t)(cn >> 2) : k;
          const int pn = inner ? fpos[(cn & 3) * NFP + m] : po;
          real qn[9];
#pragma unroll
          for (int c = 0; c < 9; ++c) qn[c] = a.q[((size_t)c * K + k2) * NP + pn];
          // jumps against the neighbour, or against the mirror state on a wall
          const bool free_wall = a.wall == 0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const real own = Qs[c * NP + po];
            jv[c] = inner ? qn[c] - own : (free_wall ? real(0) : real(-2) * own);
          }
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const real own = Qs[(3 + c) * NP + po];
            js[c] = inner ? qn[3 + c] - own : (free_wall ? real(-2) * own : real(0));
          }
        } else if (cn >= 0) {
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
        auto AnT = [&](const real* sg, real* o) {
          o[0] = sg[0] * nx + sg[5] * ny + sg[4] * nz;
          o[1] = sg[5] * nx + sg[1] * ny + sg[3] * nz;
          o[2] = sg[4] * nx + sg[3] * ny + sg[2] * nz;
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
#pragma unroll
        for (int c = 0; c < 3; ++c) Fs[c * NFP + m] = real(0.5) * ats[c] + real(0.5) * a.tau_v * atanv[c];
#pragma unroll
        for (int c = 0; c < 6; ++c) Fs[(3 + c) * NFP + m] = real(0.5) * anv[c] + real(0.5) * a.tau_s * anats[c];
      }
      wsync();
      // level 0 = L_0 F = (2N+3)/2 F + N^2/2 E E^T F in one pass, with E^T F at degree N - 1,
      //   (E^T F)_x = (1/N) [(N - |x|) F_x + (x1 + 1) F_{x+e1} + (x2 + 1) F_{x+e2}],
      //   (E y)_b = (1/N) [(N - |b|) y_b + b1 y_{b-e1} + b2 y_{b-e2}]
      for (int t = lane; t < 9 * NFP; t += 64) {
        const int c = t / NFP, b = t - c * NFP;
        int sb, b2;
        face_sb(b, sb, b2);
        const int b1 = sb - b2;
        const real* F = Fs + c * NFP;
        auto etf = [&](int x, int sx, int x2) {  // N (E^T F)_x
          return real(N - sx) * F[x] + real(sx - x2 + 1) * F[x + sx + 1] + real(x2 + 1) * F[x + sx + 2];
        };
        real e = real(0);
        if (sb < N) e += real(N - sb) * etf(b, sb, b2);
        if (b1 > 0) e += real(b1) * etf(b - sb, sb - 1, b2);
        if (b2 > 0) e += real(b2) * etf(b - sb - 1, sb - 1, b2 - 1);
        Cs[c * NP + b] = real(2 * N + 3) / real(2) * F[b] + e / real(2);  // N^2/2 (1/N) (1/N) N e
      }
      wsync();
      // level i (degree n - 1, n = N - i + 1) = (l_i / l_{i-1}) (E^{n-1}_n)^T level i-1
      int src = 0;
#pragma unroll
      for (int i = 1; i <= N; ++i) {
        const int n = N - i + 1, cnt = dim2(n - 1), dst = src + dim2(n);
        const real sc = real(lift_level(N, i) / lift_level(N, i - 1) / n);
        for (int t = lane; t < 9 * cnt; t += 64) {
          const int c = t / cnt, b = t - c * cnt;
          int sb, b2;
          face_sb(b, sb, b2);
          const int b1 = sb - b2;
          const real* C = Cs + c * NP + src;
          Cs[c * NP + dst + b] = sc * (real(n - sb) * C[b] + real(b1 + 1) * C[b + sb + 1] + real(b2 + 1) * C[b + sb + 2]);
        }
        src = dst;
        wsync();
      }
      // gather: coefficient alpha takes level alpha_f at its face multi-index
      const real fsc = gf[0];
#pragma unroll UNR
      for (int j = 0; j < L::RJ; ++j) {
        const int t = lane + 64 * j;
        if (t < 9 * NP) {
          const int c = t / NP, i = t - c * NP;
          const real g = fsc * Cs[c * NP + ((lpos[i] >> (8 * f)) & 255)];
          if constexpr (L::REG) racc[j] += g;
          else Rs[t] += g;
        }
      }
      wsync();
    }
#pragma unroll UNR
    for (int j = 0; j < L::RJ; ++j) {
      const int t = lane + 64 * j;
      if (t < 9 * NP) {
        const int c = t / NP, i = t - c * NP;
        if constexpr (L::REG) a.out[((size_t)c * K + k) * NP + i] = racc[j];
        else a.out[((size_t)c * K + k) * NP + i] = Rs[t];
      }
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
