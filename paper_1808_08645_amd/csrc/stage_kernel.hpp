// Fused BBWADG stage kernel for gfx950.
//
// One wavefront (64 lanes) owns EW consecutive elements; every intermediate lives in that
// wave's slice of LDS, so the phases below synchronise at wavefront level only. Per
// element and stage (paper eq. WADGform, Sections 4 and 5):
//   volume   : reference derivatives at degree N-1 (two coefficients per derivative),
//              combined with G = dr/dx, then one elevation back to degree N;
//   surface  : upwind/penalty flux per face coefficient (Bernstein face basis functions
//              vanish off their face, so traces are coefficient-wise), lift L^f = E_L L_0
//              with L_0 = (2N+3)/2 I + N^2/2 E E^T and layer i scaled by l_i;
//   WADG     : product with c^2_M (eq. mcoeff), M one-degree reductions, then the
//              telescoped projection (eq. telescope) with the c_j of Theorem 5.1;
//   update   : res = a res + dt rhs, q_out = q_in + b res (low-storage RK4 stage).
// The state is read from qin (own coefficients and neighbour face traces) and written to
// a different buffer, so no element can see a neighbour's updated trace.
#pragma once

#include <hip/hip_runtime.h>

#include "bbwadg_internal.hpp"

namespace bbw {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int lev_off(int N, int j) {
  int s = 0;
  for (int i = 0; i < j; ++i) s += dimp(N - i);
  return s;
}
constexpr int chain_off(int N, int i) {
  int s = 0;
  for (int l = 0; l < i; ++l) s += dim2(N - l);
  return s;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Elements per wavefront: pack small elements so that a wave's lanes are mostly busy.
template <int N>
constexpr int elems_per_wave() {
  return dimp(N) <= 32 ? 64 / dimp(N) : 1;
}

template <typename real, int N, int M, int EW>
struct StageLayout {
  static constexpr int NP = dimp(N), NP1 = dimp(N - 1), NFP = dim2(N), NFP1 = dim2(N - 1);
  static constexpr int NH = dimp(N + M), NH1 = dimp(N + M - 1), MP = dimp(M);
  static constexpr int LEV = lev_off(N, N + 1);
  // per-wave LDS slices (in reals)
  static constexpr int SQ = 0;                          // [4][EW][NP] own state
  static constexpr int SC2 = SQ + 4 * EW * NP;          // [EW][MP]
  static constexpr int SA = SC2 + EW * MP;              // volume [4][EW][NP1] | flux [2][4][EW][NFP] + [2][4][EW][NFP1]
  static constexpr int SA_SIZE = cmax(4 * EW * NP1, 8 * EW * (NFP + NFP1));
  static constexpr int SB = SA + SA_SIZE;               // lift chains [2][4][EW][NP] | WADG buffers
  static constexpr int SB_SIZE = cmax(8 * EW * NP, EW * (NH + NH1 + LEV));
  static constexpr int SR = SB + SB_SIZE;               // [EW][NP] r_p before the WADG step
  static constexpr int TOTAL = SR + EW * NP;
  static constexpr int BYTES = TOTAL * (int)sizeof(real);
  // waves per workgroup: as many as fit in 64 KiB of LDS, at most 4
  static constexpr int WPB = cmax(1, (65536 / BYTES) < 4 ? (65536 / BYTES) : 4);
};

template <typename real, int N, int M, int EW, int WPB, bool UPDATE>
__global__ __launch_bounds__(64 * WPB) void stage_kernel(const StageArgs<real> a) {
  using L = StageLayout<real, N, M, EW>;
  constexpr int NP = L::NP, NP1 = L::NP1, NFP = L::NFP, NFP1 = L::NFP1;
  constexpr int NH = L::NH, NH1 = L::NH1, MP = L::MP;
  constexpr int NS = (EW * NP + 63) / 64;  // coefficient slots per lane
  __shared__ real smem[WPB * L::TOTAL];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  real* const W = smem + wave * L::TOTAL;
  real* const sq = W + L::SQ;
  real* const sc2 = W + L::SC2;
  real* const sA = W + L::SA;
  real* const sB = W + L::SB;
  real* const sR = W + L::SR;
  const int64_t K = a.K;
  const int64_t e0 = ((int64_t)blockIdx.x * WPB + wave) * EW;
  const ushort4* const t4 = reinterpret_cast<const ushort4*>(a.tab);
  const uint16_t* const t1 = a.tab;
  const real* const qin = a.qin;

  // ---- load own state (and the RK register) -------------------------------------
  real q[4][NS], acc[4][NS], rs[4][NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int v = lane + 64 * s;
    const int e = v / NP, i = v - (v / NP) * NP;
    const int64_t k = e0 + e;
    const bool ok = (v < EW * NP) && (k < K);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const size_t g = ((size_t)f * K + k) * NP + i;
      q[f][s] = ok ? qin[g] : real(0);
      if constexpr (UPDATE) rs[f][s] = ok ? a.res[g] : real(0);
      if (v < EW * NP) sq[(f * EW + e) * NP + i] = q[f][s];
      acc[f][s] = real(0);
    }
  }
  for (int v = lane; v < EW * MP; v += 64) {
    const int e = v / MP, b = v - (v / MP) * MP;
    const int64_t k = e0 + e;
    sc2[v] = (k < K) ? a.c2[k * MP + b] : real(1);
  }
  wave_sync();

  // ---- volume: reference derivatives at degree N-1 ---------------------------------
  {
    real* const sy = sA;  // [4][EW][NP1]: -d p/dx_i (i=0..2), -div u (3), scaled by N/2
    const ushort4* up = t4 + a.off.red3[N] / 4;  // b + e_k at degree N, for b of degree N-1
    constexpr real half_n = real(N) / real(2);
    for (int v = lane; v < EW * NP1; v += 64) {
      const int e = v / NP1, b = v - (v / NP1) * NP1;
      const int64_t k = e0 + e;
      real G[9];
#pragma unroll
      for (int x = 0; x < 9; ++x) G[x] = (k < K) ? a.geo[k * kGeoStride + x] : real(0);
      const ushort4 id = up[b];
      const real* P = sq + (0 * EW + e) * NP;
      real dp[3] = {P[id.y] - P[id.x], P[id.z] - P[id.x], P[id.w] - P[id.x]};
      real div = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const real* U = sq + ((1 + i) * EW + e) * NP;
        const real u0 = U[id.x];
        div += G[3 * i + 0] * (U[id.y] - u0) + G[3 * i + 1] * (U[id.z] - u0) + G[3 * i + 2] * (U[id.w] - u0);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
        sy[(i * EW + e) * NP1 + b] = -half_n * (G[3 * i] * dp[0] + G[3 * i + 1] * dp[1] + G[3 * i + 2] * dp[2]);
      sy[(3 * EW + e) * NP1 + b] = -half_n * div;
    }
  }
  wave_sync();
  // elevate to degree N: acc[0] = -div u, acc[1+i] = -d p / d x_i
  {
    const real* const sy = sA;
    const ushort4* el = t4 + a.off.el3[N] / 4;
    const ushort4* mi = t4 + a.off.mi3[N] / 4;
    constexpr real inv_n = real(1) / real(N);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int v = lane + 64 * s;
      if (v < EW * NP) {
        const int e = v / NP, i = v - (v / NP) * NP;
        const ushort4 id = el[i];
        const ushort4 m = mi[i];
        const uint16_t ix[4] = {id.x, id.y, id.z, id.w};
        const real w[4] = {real(m.x) * inv_n, real(m.y) * inv_n, real(m.z) * inv_n, real(m.w) * inv_n};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const real* Y = sy + (c * EW + e) * NP1;
          real t = 0;
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2)
            if (ix[k2] != kNone) t += w[k2] * Y[ix[k2]];
          acc[c == 3 ? 0 : c + 1][s] = t;
        }
      }
    }
  }
  wave_sync();

  // ---- surface: fluxes per face coefficient ------------------------------------------
  real* const sF = sA;                      // [2][4][EW][NFP]
  real* const sT = sA + 8 * EW * NFP;       // [2][4][EW][NFP1]
  {
    const uint16_t* fidx = t1 + a.off.fidx;
    for (int v = lane; v < EW * 4 * NFP; v += 64) {
      const int e = v / (4 * NFP);
      const int r = v - e * (4 * NFP);
      const int f = r / NFP, m = r - (r / NFP) * NFP;
      const int64_t k = e0 + e;
      const int own = fidx[f * NFP + m];
      const real pm = sq[(0 * EW + e) * NP + own];
      const real um = sq[(1 * EW + e) * NP + own];
      const real vm = sq[(2 * EW + e) * NP + own];
      const real wm = sq[(3 * EW + e) * NP + own];
      real nx = 0, ny = 0, nz = 0;
      int32_t nb = -1;
      if (k < K) {
        const real* g = a.geo + k * kGeoStride + 9 + 4 * f;
        nx = g[1];
        ny = g[2];
        nz = g[3];
        nb = a.conn[k * 4 + f];
      }
      real pp, up, vp, wp;
      if (nb >= 0) {
        const int64_t k2 = nb >> 2;
        const int f2 = nb & 3;
        const size_t base = (size_t)k2 * NP + fidx[f2 * NFP + m];
        const size_t fs = (size_t)K * NP;
        pp = qin[base];
        up = qin[base + fs];
        vp = qin[base + 2 * fs];
        wp = qin[base + 3 * fs];
      } else if (a.bc == 0) {  // p = 0 wall: p+ = -p, u+ = u
        pp = -pm;
        up = um;
        vp = vm;
        wp = wm;
      } else {  // rigid wall: p+ = p, u+ = u - 2 (u.n) n
        const real un = um * nx + vm * ny + wm * nz;
        pp = pm;
        up = um - 2 * un * nx;
        vp = vm - 2 * un * ny;
        wp = wm - 2 * un * nz;
      }
      const real jp = pp - pm;
      const real jun = (up - um) * nx + (vp - vm) * ny + (wp - wm) * nz;
      sF[((0 * 4 + f) * EW + e) * NFP + m] = real(0.5) * (a.tau_p * jp - jun);
      sF[((1 * 4 + f) * EW + e) * NFP + m] = real(0.5) * (a.tau_u * jun - jp);
    }
  }
  wave_sync();

  // ---- lift: L_0 on each face, then the reduction chain ------------------------------
  real* const sC = sB;  // [2][4][EW][NP]: chain levels 0..N of each face flux
  {
    const ushort4* red = t4 + a.off.red2[N] / 4;
    const ushort4* mi = t4 + a.off.mi2[N - 1] / 4;
    constexpr real inv_n = real(1) / real(N);
    for (int v = lane; v < 8 * EW * NFP1; v += 64) {
      const int c = v / NFP1, b = v - (v / NFP1) * NFP1;
      const ushort4 id = red[b];
      const ushort4 m = mi[b];
      const real* F = sF + c * NFP;
      sT[c * NFP1 + b] = inv_n * (real(m.x + 1) * F[id.x] + real(m.y + 1) * F[id.y] + real(m.z + 1) * F[id.z]);
    }
  }
  wave_sync();
  {
    const ushort4* el = t4 + a.off.el2 / 4;
    const ushort4* mi = t4 + a.off.mi2[N] / 4;
    constexpr real inv_n = real(1) / real(N);
    constexpr real l0a = real(2 * N + 3) / real(2);
    constexpr real l0b = real(N * N) / real(2);
    for (int v = lane; v < 8 * EW * NFP; v += 64) {
      const int c = v / NFP, g = v - (v / NFP) * NFP;
      const ushort4 id = el[g];
      const ushort4 m = mi[g];
      const real* T = sT + c * NFP1;
      real t = 0;
      if (id.x != kNone) t += real(m.x) * T[id.x];
      if (id.y != kNone) t += real(m.y) * T[id.y];
      if (id.z != kNone) t += real(m.z) * T[id.z];
      sC[c * NP + g] = l0a * sF[c * NFP + g] + l0b * inv_n * t;
    }
  }
  wave_sync();
#pragma unroll
  for (int i = 1; i <= N; ++i) {
    const int n = N - i + 1;  // reduce degree n -> n-1
    const ushort4* red = t4 + a.off.red2[n] / 4;
    const ushort4* mi = t4 + a.off.mi2[n - 1] / 4;
    const real inv_n = real(1) / real(n);
    const int cnt = dim2(n - 1);
    const int src = chain_off(N, i - 1), dst = chain_off(N, i);
    for (int v = lane; v < 8 * EW * cnt; v += 64) {
      const int c = v / cnt, b = v - (v / cnt) * cnt;
      const ushort4 id = red[b];
      const ushort4 m = mi[b];
      const real* S = sC + c * NP + src;
      sC[c * NP + dst + b] = inv_n * (real(m.x + 1) * S[id.x] + real(m.y + 1) * S[id.y] + real(m.z + 1) * S[id.z]);
    }
    wave_sync();
  }
  // gather the four face lifts into every coefficient
  {
    const uint16_t* lpos = t1 + a.off.liftpos;
    const ushort4* mi = t4 + a.off.mi3[N] / 4;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int v = lane + 64 * s;
      if (v < EW * NP) {
        const int e = v / NP, i = v - (v / NP) * NP;
        const int64_t k = e0 + e;
        const ushort4 m = mi[i];
        const uint16_t al[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          real sc = 0, nx = 0, ny = 0, nz = 0;
          if (k < K) {
            const real* g = a.geo + k * kGeoStride + 9 + 4 * f;
            sc = g[0];
            nx = g[1];
            ny = g[2];
            nz = g[3];
          }
          const int pos = lpos[f * NP + i];
          const real ell = a.ell[al[f]] * sc;
          const real lp = sC[((0 * 4 + f) * EW + e) * NP + pos];
          const real lu = sC[((1 * 4 + f) * EW + e) * NP + pos] * ell;
          acc[0][s] += ell * lp;
          acc[1][s] += nx * lu;
          acc[2][s] += ny * lu;
          acc[3][s] += nz * lu;
        }
        if constexpr (M > 0) sR[e * NP + i] = acc[0][s];
        else acc[0][s] *= sc2[e * MP];
      }
    }
  }

  // ---- WADG: multiply by c^2_M, reduce M degrees, telescoped projection -------------
  if constexpr (M > 0) {
    wave_sync();
    real* const sH = sB;               // [EW][NH]
    real* const sH1 = sB + EW * NH;    // [EW][NH1]
    real* const sL = sH1 + EW * NH1;   // [EW][LEV] levels j = 0..N of the telescoping
    constexpr int LEV = L::LEV;
    {
      const uint16_t* mid = t1 + a.off.mulidx;
      for (int v = lane; v < EW * NH; v += 64) {
        const int e = v / NH, g = v - (v / NH) * NH;
        real h = 0;
#pragma unroll
        for (int b = 0; b < MP; ++b) {
          const uint16_t ix = mid[g * MP + b];
          if (ix != kNone) h += a.mulw[g * MP + b] * sc2[e * MP + b] * sR[e * NP + ix];
        }
        sH[e * NH + g] = h;
      }
    }
    wave_sync();
    // M reductions: degree N+M -> N (the last lands in level 0 of sL)
#pragma unroll
    for (int n = N + M; n > N; --n) {
      const int cnt = dimp(n - 1), srcn = dimp(n);
      const real* src = ((N + M - n) % 2 == 0) ? sH : sH1;
      real* dst = (n - 1 == N) ? sL : (((N + M - n) % 2 == 0) ? sH1 : sH);
      const int dstride = (n - 1 == N) ? LEV : cnt;
      const ushort4* red = t4 + a.off.red3[n] / 4;
      const ushort4* mi = t4 + a.off.mi3[n - 1] / 4;
      const real inv_n = real(1) / real(n);
      for (int v = lane; v < EW * cnt; v += 64) {
        const int e = v / cnt, b = v - (v / cnt) * cnt;
        const ushort4 id = red[b];
        const ushort4 m = mi[b];
        const real* S = src + e * srcn;
        dst[e * dstride + b] = inv_n * (real(m.x + 1) * S[id.x] + real(m.y + 1) * S[id.y] +
                                         real(m.z + 1) * S[id.z] + real(m.w + 1) * S[id.w]);
      }
      wave_sync();
    }
    // downward sweep: level j = (E^{N-j+1}_{N-j})^T level j-1
#pragma unroll
    for (int j = 1; j <= N; ++j) {
      const int n = N - j + 1;
      const int cnt = dimp(n - 1);
      const ushort4* red = t4 + a.off.red3[n] / 4;
      const ushort4* mi = t4 + a.off.mi3[n - 1] / 4;
      const real inv_n = real(1) / real(n);
      const int src = lev_off(N, j - 1), dst = lev_off(N, j);
      for (int v = lane; v < EW * cnt; v += 64) {
        const int e = v / cnt, b = v - (v / cnt) * cnt;
        const ushort4 id = red[b];
        const ushort4 m = mi[b];
        const real* S = sL + e * LEV + src;
        sL[e * LEV + dst + b] = inv_n * (real(m.x + 1) * S[id.x] + real(m.y + 1) * S[id.y] +
                                         real(m.z + 1) * S[id.z] + real(m.w + 1) * S[id.w]);
      }
      wave_sync();
    }
    // upward sweep: s_N = c_N r_N; s_j = c_j r_j + E^{N-j}_{N-j-1} s_{j+1}
    for (int v = lane; v < EW; v += 64) sL[v * LEV + lev_off(N, N)] *= a.cj[N];
    wave_sync();
#pragma unroll
    for (int j = N - 1; j >= 0; --j) {
      const int n = N - j;  // degree of level j
      const int cnt = dimp(n);
      const ushort4* el = t4 + a.off.el3[n] / 4;
      const ushort4* mi = t4 + a.off.mi3[n] / 4;
      const real inv_n = real(1) / real(n);
      const real cj = a.cj[j];
      const int lo = lev_off(N, j), hi = lev_off(N, j + 1);
      for (int v = lane; v < EW * cnt; v += 64) {
        const int e = v / cnt, g = v - (v / cnt) * cnt;
        const ushort4 id = el[g];
        const ushort4 m = mi[g];
        const real* S = sL + e * LEV + hi;
        real t = 0;
        if (id.x != kNone) t += real(m.x) * S[id.x];
        if (id.y != kNone) t += real(m.y) * S[id.y];
        if (id.z != kNone) t += real(m.z) * S[id.z];
        if (id.w != kNone) t += real(m.w) * S[id.w];
        real* D = sL + e * LEV + lo + g;
        *D = cj * (*D) + inv_n * t;
      }
      wave_sync();
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int v = lane + 64 * s;
      if (v < EW * NP) {
        const int e = v / NP, i = v - (v / NP) * NP;
        acc[0][s] = sL[e * LEV + i];
      }
    }
  }

  // ---- write: rhs, or the low-storage RK stage ----------------------------------------
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int v = lane + 64 * s;
    const int e = v / NP, i = v - (v / NP) * NP;
    const int64_t k = e0 + e;
    if (v < EW * NP && k < K) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const size_t g = ((size_t)f * K + k) * NP + i;
        if constexpr (UPDATE) {
          const real r = a.rk_a * rs[f][s] + a.dt * acc[f][s];
          a.res[g] = r;
          a.qout[g] = q[f][s] + a.rk_b * r;
        } else {
          a.qout[g] = acc[f][s];
        }
      }
    }
  }
}

template <typename real, int N, int M, bool UPDATE>
int launch_stage_typed(const StageArgs<real>& a, void* stream) {
  constexpr int EW = elems_per_wave<N>();
  using L = StageLayout<real, N, M, EW>;
  constexpr int WPB = L::WPB;
  const int64_t per_block = (int64_t)EW * WPB;
  const int64_t blocks = (a.K + per_block - 1) / per_block;
  if (blocks <= 0) return 0;
  hipLaunchKernelGGL((stage_kernel<real, N, M, EW, WPB, UPDATE>), dim3((unsigned)blocks), dim3(64 * WPB), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

// Per-field squared L^2 norms with the closed-form Bernstein mass matrix, FP64
// accumulation: one wave per element, lane i forms q_i (M q)_i, block partials.
template <typename real, int N>
__global__ __launch_bounds__(256) void l2norm_kernel(const real* q, int64_t K, const double* J,
                                                     const double* mass, double* partial) {
  constexpr int NP = dimp(N);
  constexpr int NS = (NP + 63) / 64;
  __shared__ double sv[4][4][NP];
  __shared__ double red[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double accf[4] = {0, 0, 0, 0};
  for (int64_t k = (int64_t)blockIdx.x * 4 + wave; k < K; k += (int64_t)gridDim.x * 4) {
    for (int f = 0; f < 4; ++f)
      for (int i = lane; i < NP; i += 64) sv[wave][f][i] = (double)q[((size_t)f * K + k) * NP + i];
    wave_sync();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + 64 * s;
      if (i < NP) {
        for (int f = 0; f < 4; ++f) {
          double t = 0;
          for (int j = 0; j < NP; ++j) t += mass[i * NP + j] * sv[wave][f][j];
          accf[f] += J[k] * sv[wave][f][i] * t;
        }
      }
    }
    wave_sync();
  }
  for (int f = 0; f < 4; ++f) {
    double v = accf[f];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave][f] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int f = threadIdx.x;
    partial[blockIdx.x * 4 + f] = red[0][f] + red[1][f] + red[2][f] + red[3][f];
  }
}

template <typename real, int N>
int launch_l2norm_typed(const void* q, int64_t K, const double* J, const double* mass, double* partial,
                        int nblocks, void* stream) {
  hipLaunchKernelGGL((l2norm_kernel<real, N>), dim3(nblocks), dim3(256), 0, (hipStream_t)stream,
                     (const real*)q, K, J, mass, partial);
  return (int)hipGetLastError();
}

}  // namespace bbw

namespace bbw {

template <int N, int M>
int dispatch_nm(bool update, bool f64, const void* args, void* stream) {
  if (f64) {
    const auto& a = *static_cast<const StageArgs<double>*>(args);
    return update ? launch_stage_typed<double, N, M, true>(a, stream) : launch_stage_typed<double, N, M, false>(a, stream);
  }
  const auto& a = *static_cast<const StageArgs<float>*>(args);
  return update ? launch_stage_typed<float, N, M, true>(a, stream) : launch_stage_typed<float, N, M, false>(a, stream);
}

// All c^2 degrees M <= min(N, kMaxM) of one polynomial degree N.
template <int N>
int launch_stage_degree(int M, bool update, bool f64, const void* args, void* stream) {
  switch (M) {
    case 0: return dispatch_nm<N, 0>(update, f64, args, stream);
    case 1: if constexpr (N >= 1) return dispatch_nm<N, 1>(update, f64, args, stream); break;
    case 2: if constexpr (N >= 2) return dispatch_nm<N, 2>(update, f64, args, stream); break;
    case 3: if constexpr (N >= 3) return dispatch_nm<N, 3>(update, f64, args, stream); break;
    case 4: if constexpr (N >= 4) return dispatch_nm<N, 4>(update, f64, args, stream); break;
    default: break;
  }
  return (int)hipErrorInvalidValue;
}

template <int N>
int launch_l2norm_degree(bool f64, const void* q, int64_t K, const double* J, const double* mass, double* partial,
                         int nblocks, void* stream) {
  return f64 ? launch_l2norm_typed<double, N>(q, K, J, mass, partial, nblocks, stream)
             : launch_l2norm_typed<float, N>(q, K, J, mass, partial, nblocks, stream);
}

}  // namespace bbw

// One translation unit per degree N keeps compile units small and parallel.
#define BBW_DEGREE_UNIT(NN)                                                                                    \
  namespace bbw {                                                                                              \
  int launch_stage_n##NN(int M, bool update, bool f64, const void* args, void* stream) {                      \
    return launch_stage_degree<NN>(M, update, f64, args, stream);                                              \
  }                                                                                                            \
  int launch_l2norm_n##NN(bool f64, const void* q, int64_t K, const double* J, const double* mass,            \
                          double* partial, int nblocks, void* stream) {                                        \
    return launch_l2norm_degree<NN>(f64, q, K, J, mass, partial, nblocks, stream);                             \
  }                                                                                                            \
  }
