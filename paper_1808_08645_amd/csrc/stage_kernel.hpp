// Fused BBWADG stage kernel for gfx950.
//
// One stage of the method for every element (paper eq. WADGform, Sections 4 and 5):
//   volume  : reference derivatives at degree N-1 (two coefficients each), combined with
//             G = dr/dx, then one degree elevation back to N (Section 4);
//   surface : penalty flux per face coefficient (Bernstein face functions vanish off their
//             face, so traces are coefficient-wise), lift L^f = E_L L_0 with
//             L_0 = (2N+3)/2 I + N^2/2 E E^T and layer i scaled by l_i (Section 4);
//   WADG    : product with c^2_M (eq. mcoeff), M one-degree reductions and the telescoped
//             projection (eq. telescope) with the c_j of Theorem 5.3 (Section 5);
//   update  : res = a res + dt rhs, q_out = q_in + b res (low-storage RK4 stage).
//
// Design for CDNA4:
// * Coefficients use a graded order (by a1+a2+a3), so the degree-n coefficient list is a
//   prefix of the degree-(n+1) list and a lane keeps the same multi-index at every
//   degree. Each lane therefore computes its stencil neighbours (alpha +- e_k, face maps,
//   lift positions, product positions) once, into registers; the element loop reads no
//   index table.
// * A wavefront owns EW elements at a time and keeps every intermediate in its own slice
//   of LDS; phases synchronise at wavefront level only. Since a lane holds the same
//   position at every degree, each stencil's own-position term is taken from the lane's
//   registers and only neighbour terms are read from LDS.
// * The WADG levels are kept scaled by a1!a2!a3! (reductions) or its inverse (elevations),
//   which leaves a single weight per stencil.
// * Waves are persistent: each XCD processes a contiguous range of elements so that face
//   neighbours are found in that XCD's L2, and the next element group's state, geometry
//   and c^2 are prefetched into registers while the current one is computed.
// * The state is read from qin and the next state written to qout (a different buffer),
//   so no element ever reads a neighbour's updated trace.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>

#include "bbwadg_internal.hpp"

namespace bbw {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// An opaque copy: the compiler may neither hoist work derived from it out of a loop nor
// share such work between uses (recomputing a few integer ops beats holding registers).
__device__ __forceinline__ int opq(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Load through the constant address space: with a wave-uniform address this is a scalar
// load into SGPRs (per-element data of a team that owns one element).
template <typename T>
__device__ __forceinline__ T uload(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}
// The value of v in lane l of the wavefront (l uniform), as a scalar.
template <typename T>
__device__ __forceinline__ T lane_value(T v, int l) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// Graded position of (a1, a2, a3): dimp(s-1) + a3 (2s+3-a3)/2 + a2, s = a1+a2+a3.
__host__ __device__ constexpr int g3(int a1, int a2, int a3) {
  return dimp(a1 + a2 + a3 - 1) + a3 * (2 * (a1 + a2 + a3) + 3 - a3) / 2 + a2;
}
// Graded face position of (b1, b2): t(t+1)/2 + b2, t = b1+b2.
__host__ __device__ constexpr int g2(int b1, int b2) { return (b1 + b2) * (b1 + b2 + 1) / 2 + b2; }

// Start of level i (degree N-i) in a concatenated face chain.
constexpr int chain_off(int N, int i) {
  int s = 0;
  for (int l = 0; l < i; ++l) s += dim2(N - l);
  return s;
}
// Start of level j (degree N-j) in the concatenated telescoping levels. Levels j >= 1 are
// preceded by one position that stays zero: an elevation reads it for a missing neighbour.
constexpr int lev_off(int N, int j) {
  int s = 0;
  for (int i = 0; i < j; ++i) s += dimp(N - i) + 1;
  return s;
}
__host__ __device__ constexpr long long fact(int n) {
  long long r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}
__host__ __device__ constexpr long long binom(int n, int k) {
  return (k < 0 || k > n) ? 0 : fact(n) / (fact(k) * fact(n - k));
}
// l_i = (-1)^i C(N, i) / (i + 1): factor of lift layer i.
__host__ __device__ constexpr double lift_ell(int N, int i) { return (i % 2 ? -1.0 : 1.0) * (double)binom(N, i) / (double)(i + 1); }

// Multi-index of graded position p: (a1, a2, a3).
__device__ inline void pos3(int p, int& a1, int& a2, int& a3) {
  int s = 0;
  while (dimp(s) <= p) ++s;
  int r = p - dimp(s - 1);
  int c = 0;
  while (r >= s - c + 1) {
    r -= s - c + 1;
    ++c;
  }
  a3 = c;
  a2 = r;
  a1 = s - r - c;
}
__device__ inline void pos2(int p, int& b1, int& b2) {
  int t = 0;
  while ((t + 1) * (t + 2) / 2 <= p) ++t;
  b2 = p - t * (t + 1) / 2;
  b1 = t - b2;
}

// Elements per team: pack small elements so that most lanes are busy.
template <int N>
constexpr int elems_per_wave() {
  return dimp(N) <= 32 ? 64 / dimp(N) : 1;
}
// Waves per team: large elements are shared by up to four wavefronts so that each lane
// carries at most a few coefficients.
template <int N>
constexpr int waves_per_team() {
  return dimp(N) <= 64 ? 1 : (dimp(N) + 63) / 64 > 4 ? 4 : (dimp(N) + 63) / 64;
}

// How a group's global loads are placed around its phases:
//   kLoadsEarly : neighbour traces and the next group's state/geometry/c^2 requested at the
//                 top (registers), the RK register after the flux phase (registers);
//   kLoadsLate  : neighbour traces requested just before the flux phase, the next group's
//                 data after it (registers; fewer registers held through the volume phases);
//   kLoadsLds   : neighbour traces one group ahead and the RK register straight into LDS
//                 (no registers for them; one-wave teams only), the next group's data after
//                 the flux phase.
// The choice per degree and precision is the measured fastest (BBW_LOADS forces one).
enum { kLoadsEarly = 0, kLoadsLate = 1, kLoadsLds = 2 };
#ifndef BBW_LOADS
#define BBW_LOADS -1
#endif
// Measured (196,608 tets, M = N/2, ms per stage, early / late / LDS): FP64 N=5 0.467 / 0.489 /
// 0.481, N=6 0.926 / 0.949, N=7 1.74 / 1.42, N=8 4.16 / 2.49, N=9 4.58 / 3.46; FP32 within 2%
// of each other at N <= 4 and early fastest from N = 5 (0.272 / 0.278 / 0.281 at N = 5; N = 6
// to 9 early / late 0.552 / 0.566, 0.809 / 0.841, 1.647 / 1.704, 2.239 / 2.307).
constexpr int loads_table(int bytes, int N, int TW) {
  (void)TW;
  return (bytes == 8 && N >= 7) ? kLoadsLate : kLoadsEarly;
}
template <typename real, int N, int TW>
constexpr int stage_loads() {
  if (BBW_LOADS >= 0) return (BBW_LOADS == kLoadsLds && TW > 1) ? kLoadsLate : BBW_LOADS;
  return loads_table((int)sizeof(real), N, TW);
}

// Product positions are kept in registers when MP * S3 is at most this, else derived per use.
#ifndef BBW_MUL_REGS_MAX
#define BBW_MUL_REGS_MAX 40
#endif

// Face-chain layout: unpadded rows with the channel XOR-swizzled by the row (1), or an odd
// row pitch (0).
#ifndef BBW_CHAIN_SWZ
#define BBW_CHAIN_SWZ 1
#endif

template <typename real, int N, int M, int EW>
struct StageLayout {
  static constexpr int TW = waves_per_team<N>();     // waves per team (one team owns EW elements)
  static constexpr int TL = 64 * TW;                   // lanes per team
  static constexpr int NP = dimp(N), NP1 = dimp(N - 1), NFP = dim2(N), NFP1 = dim2(N - 1);
  static constexpr int NH = dimp(N + M), NH1 = dimp(N + M - 1), MP = dimp(M);
  static constexpr int LEV = lev_off(N, N + 1);
  // FP32 state with the telescoping in FP64 where the c_j amplify rounding most
  // (N >= BBW_TELE64_MIN_N); the levels are then doubles (+ 2 reals: 8-byte aligned start)
  static constexpr bool TELE64 = sizeof(real) == 4 && N >= BBW_TELE64_MIN_N && M > 0;
  static constexpr int LEVA = TELE64 ? 2 * LEV + 2 : LEV;
  static constexpr int PW = 25 + MP;                   // per-element scalars: geometry + c^2
  static constexpr int S3 = cdiv(EW * NH, TL);         // 3D slots (degree <= N+M)
  static constexpr int S3N = cdiv(EW * NP, TL);        // 3D slots covering degree N
  static constexpr int S2 = cdiv(8 * EW * NFP, TL);    // face-chain slots (8 channels per element)
  static constexpr int SF = cdiv(4 * EW * NFP, TL);    // flux slots (4 faces per element)
  static constexpr int SPW = cdiv(EW * PW, TL);        // per-element scalar loads per lane
  static constexpr int CH = 8 * EW;                    // chain channels: (p, u) x 4 faces x EW
  // Face-chain arrays hold one real per unit b*CHP + slot(b, channel). With a power-of-two
  // channel count the rows are unpadded and the channel is XOR-swizzled by the low bits of
  // the row, so that lanes reading one channel from different rows spread over the banks
  // while a row stays one contiguous run; otherwise the row pitch is odd.
  static constexpr bool SWZ = BBW_CHAIN_SWZ && (CH & (CH - 1)) == 0;
  static constexpr int CHP = SWZ ? CH : (CH % 2 ? CH : CH + 1);
  static __host__ __device__ constexpr int cunit(int row, int ch) { return row * CHP + (SWZ ? (ch ^ (row & 7)) : ch); }
  // Per-wave LDS slice, in reals. A 3D array holds one real per unit pos*EW + e; a field
  // array is 4 such planes.
  static constexpr int OFF_P = 0;                          // [EW][25] geometry, [EW][MP] c^2/beta!
  static constexpr int OFF_Q = cdiv(EW * PW, 2) * 2;       // 4 planes [NP*EW] state
  static constexpr int PLQ = EW * NP;
  static constexpr int OFF_A = cdiv(OFF_Q + 4 * PLQ, 8) * 8;  // Y: 4 planes [NP1*EW] | F [NFP*CHP], T [NFP1*CHP] | R [NP*EW]
  static constexpr int PLY = EW * NP1;
  static constexpr int SA = cmax(4 * PLY + EW * (NP - NP1), CHP * (NFP + NFP1));
  static constexpr int OFF_B = cdiv(OFF_A + SA, 8) * 8;    // chain [NP*CHP] | H, H1, levels
  static constexpr int SB = cmax(CHP * NP, EW * (NH + NH1 + LEVA) + 4 * EW);  // LEV includes the level guards
  static constexpr int OFF_Z = OFF_B + SB;                 // a real that stays zero
  static constexpr int TOTAL = cdiv(OFF_Z + 2, 8) * 8;  // slices stay 8-real aligned
  // direct-load buffer (dwords per team): the RK register [4][S3N] of the group, each real
  // as sizeof(real)/4 dwords of TL lanes. One-wave teams only: a multi-wave team's buffer
  // would cost more occupancy (LDS) than its registers do.
  static constexpr int LOADS = stage_loads<real, N, TW>();
  static constexpr bool RS_DMA = LOADS == kLoadsLds;
  static constexpr int NH2 = (int)sizeof(real) / 4;
  // ... and, before it, the neighbour traces: [4 fields][NH2 halves] x the rows of the SF flux
  // slots, a row as wide as its items (the last rounded up to 32 lanes), requested one group
  // ahead
  static constexpr int NBLAST = cdiv(4 * EW * NFP - TL * (SF - 1), 32) * 32;  // last row's width
  static constexpr int NBR = TL * (SF - 1) + NBLAST;                         // one field-half
  static constexpr int NBW = RS_DMA ? 4 * NH2 * NBR : 0;
  static constexpr int DBW = RS_DMA ? NBW + 4 * S3N * NH2 * TL : 0;
  static constexpr int BYTES = TOTAL * (int)sizeof(real) + 4 * DBW;
  // teams per workgroup: single-wave teams share a workgroup (up to 4 within 64 KiB of LDS);
  // a multi-wave team is a workgroup of its own, synchronised by the workgroup barrier
  static constexpr int TPB = TW > 1 ? 1 : cmax(1, (65536 / BYTES) < 4 ? (65536 / BYTES) : 4);
  static constexpr int WPB = TW * TPB;
  // product positions kept in registers when they are few, read from the byte table
  // otherwise. FP64 N = 6, M = 3 (40 positions) takes the table: its 20 position registers
  // held the instance at 184 VGPRs (2 waves per SIMD); with the table it has 149 (3 waves)
  // and runs 0.942 against 1.047 ms per stage at 196,608 tets. Elsewhere the registers
  // measured faster (FP64 N = 5, M = 2: 0.460 against 0.488; FP32 N = 6, M = 3: 0.550
  // against 0.623).
  static constexpr bool MUL_REGS = MP * S3 <= BBW_MUL_REGS_MAX && !(sizeof(real) == 8 && N == 6 && M == 3);
  static constexpr int PTAB_BYTES = MUL_REGS ? 1 : MP * EW * NH;
  // waves per SIMD that LDS allows (160 KiB per CU, 4 SIMDs); registers are budgeted for
  // the same occupancy, at most 4
  static constexpr int LDS_WAVES = (163840 / (BYTES * TPB + PTAB_BYTES)) * WPB / 4;
  static constexpr int WAVES_EU = LDS_WAVES < 1 ? 1 : (LDS_WAVES > 4 ? 4 : LDS_WAVES);
};

// Volume position of face coefficient (b0, b1, b2) of face f (face f is opposite local
// vertex f; its vertices in increasing order carry b0, b1, b2).
__device__ inline int face_pos(int f, int b0, int b1, int b2) {
  switch (f) {
    case 0: return g3(b0, b1, b2);
    case 1: return g3(0, b1, b2);
    case 2: return g3(b1, 0, b2);
    default: return g3(b1, b2, 0);
  }
}


// Which phases take their own-position ("self") term from registers instead of LDS: bit 0
// the volume's state, bit 1 the derivative planes, bit 2 the face chain, bit 3 the WADG
// levels.
#ifndef BBW_CARRY
#define BBW_CARRY 15
#endif

// Per-element scalars (geometry, c^2) of a one-element team: from the LDS copy (0), through
// scalar loads (1), read across lanes from the register that staged them (2), or geometry
// by lane reads and the c^2 coefficients by one batch of scalar loads at the start of the
// product (3). Scalar loads share their wait counter with LDS reads and return out of
// order, so every use of one waits for all LDS reads in flight; a lane read (v_readlane)
// waits for nothing but is a vector instruction, and the product reads each coefficient
// once per slot. BBW_SGPR_ELEM >= 0 overrides the table.
#ifndef BBW_SGPR_ELEM
#define BBW_SGPR_ELEM -1
#endif
// Product terms per batch of the table-driven product (each batch's reads are in flight
// together, and its sum is formed before the next batch's reads are issued, which bounds
// the registers they hold). BBW_PROD_BATCH > 0 overrides the table.
#ifndef BBW_PROD_BATCH
#define BBW_PROD_BATCH 0
#endif
// Measured at 196,608 tets, M = N/2, ms per stage. Against scalar loads with one product
// term at a time (the earlier form): FP64 N = 7 scalar loads, batches of 2: 1.374 (1.425);
// N = 8 lane reads, 8: 2.158 (2.501; scalar loads 3.40); N = 9 scalar loads, 8: 3.070
// (3.473; lane reads 3.94); FP32 N = 7, 8, 9, 8: 0.813, 1.665, 2.313 (0.921, 2.134, 2.921).
// Mode 3 against those: FP64 N = 4 0.313 (0.319), N = 5 0.458 (0.461, lane reads; 0.470
// scalar loads), N = 6 0.924 (0.943, scalar loads), N = 7 1.329 (1.370), N = 9 2.985
// (3.065); FP32 N = 9 2.235 (2.298), the rest within 1%. Batches of 4 for FP64 N = 7 and 8
// (with mode 3): 1.250 and 2.112 against 1.335 (2; 1.534 with 8) and 2.154 (8); FP64 N = 6
// and 9 and FP32 N = 7..9 are fastest with 8 (FP64 N = 6 with scalar loads: 0.943 / 0.956 /
// 1.001 with 8 / 4 / 2).
constexpr int batch_table(int bytes, int N) { return bytes == 8 && (N == 7 || N == 8) ? 4 : 8; }
template <typename real, int N>
constexpr int stage_scalars() { return BBW_SGPR_ELEM >= 0 ? BBW_SGPR_ELEM : 3; }  // mode 3 at every degree
template <typename real, int N>
constexpr int stage_batch() { return BBW_PROD_BATCH > 0 ? BBW_PROD_BATCH : batch_table((int)sizeof(real), N); }

// Optional occupancy target (waves per SIMD) for the register allocator; 0 leaves the
// choice to the compiler (or to the per-instance targets below).
#ifndef BBW_WAVES_EU
#define BBW_WAVES_EU 0
#endif

#ifndef BBW_F32_TARGET4
#define BBW_F32_TARGET4 0
#endif

// Instances whose register allocation is steered to 3 waves per SIMD: there the compiler's
// own choice lands just above the 168 registers that 3 waves allow, and the target is met
// without spilling (FP64 at N = 5, M <= 2 and N = 7, M = 2; LDS allows it).
template <typename real, int N, int M>
constexpr int stage_waves_target() {
  if (BBW_WAVES_EU > 0) return BBW_WAVES_EU;
  if (sizeof(real) == 8) return ((N == 5 && M <= 2) || (N == 7 && M == 2)) ? 3 : 0;
  return (BBW_F32_TARGET4 && N == 5 && M <= 2) ? 4 : 0;
}

template <typename real, int N, int M, int EW, int WPB, bool UPDATE, bool RPOUT = false>
__global__ __launch_bounds__(64 * WPB)
__attribute__((amdgpu_waves_per_eu(
    stage_waves_target<real, N, M>() > 0 && stage_waves_target<real, N, M>() <= StageLayout<real, N, M, EW>::WAVES_EU
        ? stage_waves_target<real, N, M>() : 1, 8)))
void stage_kernel(const StageArgs<real> a) {
  using L = StageLayout<real, N, M, EW>;
  constexpr int NP = L::NP, NP1 = L::NP1, NFP = L::NFP, NFP1 = L::NFP1, NH = L::NH, MP = L::MP;
  constexpr int S3 = L::S3, S3N = L::S3N, S2 = L::S2, SF = L::SF, SPW = L::SPW, PW = L::PW;
  constexpr int CH = L::CH, CHP = L::CHP;
  constexpr int TW = L::TW, TL = L::TL, TPB = L::TPB;
  constexpr int SZ = (int)sizeof(real);
  // byte offsets of the arrays inside a wave's slice
  constexpr int BP = L::OFF_P * SZ, BQ = L::OFF_Q * SZ, BA = L::OFF_A * SZ, BB = L::OFF_B * SZ;
  constexpr int BZ = L::OFF_Z * SZ;
  constexpr int PQ = L::PLQ * SZ, PY = L::PLY * SZ;  // plane strides
  __shared__ __attribute__((aligned(16))) real smem[TPB * L::TOTAL];
  // The RK register of the group arrives by direct global-to-LDS loads (no registers while
  // the lift and the weight adjustment run): one dword per lane and instruction, in
  // [field][slot][half][team lane] dword order (a real is one or two dwords, its halves TL
  // dwords apart). The compiler waits for all outstanding memory operations before this
  // array is read, so it is requested late (after the flux phase) and read at the very end,
  // when the loads issued with it have long arrived.
  constexpr int NH2 = L::NH2, DBW = L::DBW;
  __shared__ __attribute__((aligned(16))) uint32_t dbuf[TPB * DBW + 1];
  // Without product positions in registers, a block-wide table holds pos(gamma - beta) for
  // every beta and product item (one byte each; NP marks a term that does not exist and
  // reads the zero cell after R).
  constexpr int PTAB = L::PTAB_BYTES;
  __shared__ uint8_t ptab[PTAB];
  static_assert(L::MUL_REGS || NP < 256, "positions must fit a byte");
  char* const lds = reinterpret_cast<char*>(smem);
  auto at = [lds](int byteoff) -> real& { return *reinterpret_cast<real*>(lds + byteoff); };

  const int lane = threadIdx.x % TL;  // lane within the team
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / TL);
  const int wb = team * L::TOTAL * SZ;  // this team's slice
  auto team_sync = [] {
    if constexpr (TW == 1) wave_sync();
    else __syncthreads();
  };
  const int64_t K = a.K;
  const real* const qin = a.qin;
  // direct loads into the team's dbuf rows: row dw (uniform) gets, at team lane l, dword h of
  // the real at src of lane l; lds_real reads the lane's real back from its row
  const int wl0 = __builtin_amdgcn_readfirstlane(lane & ~63);  // first team lane of this wave
  auto dma = [&](uint32_t* buf, int dw, const real* src, int h) {
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const char*>(src) + 4 * h,
                                     (__attribute__((address_space(3))) void*)(buf + dw + wl0), 4, 0, 0);
  };
  auto lds_real = [&](const uint32_t* buf, int dw, int half_stride) -> real {
    if constexpr (SZ == 4) {
      return __builtin_bit_cast(real, buf[dw + lane]);
    } else {
      const uint64_t v = (uint64_t)buf[dw + lane] | ((uint64_t)buf[dw + half_stride + lane] << 32);
      return __builtin_bit_cast(real, v);
    }
  };
  uint32_t* const nbt = dbuf + team * DBW;   // neighbour traces (one-wave teams)
  uint32_t* const rbt = nbt + L::NBW;        // RK register (one-wave teams)

  // ---- which element groups this wave owns: contiguous ranges per XCD ----------------
  const int64_t ngroups = (K + EW - 1) / EW;
  const int nxcd = (gridDim.x % 8 == 0) ? 8 : 1;
  const int xcd = blockIdx.x % nxcd;
  const int64_t waves_per_xcd = (int64_t)(gridDim.x / nxcd) * TPB;  // teams per XCD
  const int64_t lw = (int64_t)(blockIdx.x / nxcd) * TPB + team;
  const int64_t chunk = (ngroups + nxcd - 1) / nxcd;
  const int64_t gbeg = xcd * chunk;
  const int64_t gend = gbeg + chunk < ngroups ? gbeg + chunk : ngroups;

  // ---- per-lane index registers (computed once) -------------------------------------
  // 3D slot s holds unit lane + 64 s = pos*EW + e, pos the graded position of (a1,a2,a3).
  // Stencil neighbours follow from the graded order:
  //   pos(a+e1) = pos + D(s) + a3, pos(a+e2) = pos + D(s) + a3 + 1, pos(a+e3) = pos + D(s) + s + 2
  // with D(s) = (s+1)(s+2)/2 and s = a1+a2+a3 (and the same relations read backwards).
  int pa3[S3];
  // fac3 = 1/alpha!, facH = gamma! A(gamma) / C(N+M, N), aF = A(alpha) and iA2 = 1/A(alpha)^2
  // with A(alpha) = a1! a2! a3!: the WADG levels are kept scaled by A (reductions) or by
  // 1/A (elevations), which leaves one weight per stencil.
  real fac3[S3N], facH[S3], aF[S3N], iA2[S3N];
  double iA2d[L::TELE64 ? S3N : 1];  // 1/A^2 in FP64 (FP64 telescoping)
  // product positions, two 16-bit byte offsets per register
  int mpos[L::MUL_REGS ? S3 : 1][L::MUL_REGS ? (MP + 1) / 2 : 1];
#pragma unroll
  for (int s = 0; s < S3; ++s) {
    const int item = lane + TL * s;
    const int pos = item / EW, e = item - (item / EW) * EW;
    int a1 = 0, a2 = 0, a3 = 0;
    if (item < EW * NH) pos3(pos, a1, a2, a3);
    const int sa = a1 + a2 + a3;
    pa3[s] = a1 | (a2 << 8) | (a3 << 16) | (sa << 24);
    const int a0N = N - sa, a0H = N + M - sa;
    const double Af = double(fact(a1) * fact(a2) * fact(a3));
    facH[s] = real(double(fact(a0H)) * Af * Af / double(binom(N + M, N)));
    if (s < S3N) {
      const int sN = s < S3N ? s : 0;
      fac3[sN] = (a0N >= 0) ? real(1) / real(fact(a0N) * fact(a1) * fact(a2) * fact(a3)) : real(0);
      aF[sN] = real(Af);
      iA2[sN] = real(1.0 / (Af * Af));
      if constexpr (L::TELE64) iA2d[sN] = 1.0 / (Af * Af);
    }
    if constexpr (L::MUL_REGS) {
      int b = 0;  // beta in the graded coefficient order of c^2
#pragma unroll
      for (int sb = 0; sb <= M; ++sb)
#pragma unroll
        for (int b3 = 0; b3 <= sb; ++b3)
#pragma unroll
          for (int b2 = 0; b2 <= sb - b3; ++b2) {
            const int b1 = sb - b2 - b3, b0 = M - sb;
            const bool ok = a1 >= b1 && a2 >= b2 && a3 >= b3 && a0H >= b0;
            const int off = wb + (ok ? BA + (g3(a1 - b1, a2 - b2, a3 - b3) * EW + e) * SZ : BZ);
            if (b % 2 == 0) mpos[s][b / 2] = off;
            else mpos[s][b / 2] |= off << 16;
            ++b;
          }
    }
  }
  // face-chain slot t holds item b*CH + ch (b the graded face position of (b1, b2)),
  // stored at unit b*CHP + ch; neighbours: pos(b+e1) = pos + t + 1, pos(b+e2) = pos + t + 2
  int pb2[S2];
#pragma unroll
  for (int t = 0; t < S2; ++t) {
    const int item = lane + TL * t;
    int b1 = 0, b2 = 0;
    if (item < CH * NFP) pos2(item / CH, b1, b2);
    pb2[t] = b1 | (b2 << 8) | ((b1 + b2) << 16);
  }
  // flux slot u holds face coefficient m of face f of element e (unit m*4EW + f*EW + e)
  int fown[SF], fnb[SF], ffe[SF];
#pragma unroll
  for (int u = 0; u < SF; ++u) {
    const int item = lane + TL * u;
    const int m = item / (4 * EW), fe = item - (item / (4 * EW)) * (4 * EW);
    const int f = fe / EW, e = fe - (fe / EW) * EW;
    int b1 = 0, b2 = 0;
    if (item < 4 * EW * NFP) pos2(m, b1, b2);
    const int b0 = N - b1 - b2;
    fown[u] = wb + (face_pos(f, b0, b1, b2) * EW + e) * SZ;
    // the same face coefficient seen from a neighbour's face f2 (four 8-bit positions)
    fnb[u] = face_pos(0, b0, b1, b2) | (face_pos(1, b0, b1, b2) << 8) | (face_pos(2, b0, b1, b2) << 16) |
             (face_pos(3, b0, b1, b2) << 24);
    ffe[u] = fe | (m << 16);
  }
  // Neighbour offsets (bytes, this team's slice), computed once and kept in registers;
  // weights are recomputed per phase from an opaque copy of the packed multi-index, so that
  // the compiler does not hold one converted weight per phase and slot.
  int o3p[S3][7], o2p[S2][5];
  int o3[7];
#pragma unroll
  for (int s = 0; s < S3; ++s) {
    const int p = pa3[s];
    const int a1 = p & 255, a3 = (p >> 16) & 255, sa = p >> 24, a2 = (p >> 8) & 255;
    const int self = wb + (lane + TL * s) * SZ;
    const int du = ((sa + 1) * (sa + 2) >> 1) * EW * SZ;  // D(s)
    const int dd = ((sa * (sa + 1)) >> 1) * EW * SZ;      // D(s-1)
    o3[0] = self;
    o3[1] = self + du + a3 * EW * SZ;
    o3[2] = o3[1] + EW * SZ;
    o3[3] = self + du + (sa + 2) * EW * SZ;
    // a missing neighbour (a_k = 0) is position -1 of the array read: the zero guard in
    // front of a telescoping level, a finite value elsewhere (where its weight is zero)
    const int e = (lane + TL * s) - ((lane + TL * s) / EW) * EW;
    const int none = wb + (e - EW) * SZ;
    o3[4] = a1 > 0 ? self - dd - a3 * EW * SZ : none;
    o3[5] = a2 > 0 ? self - dd - (a3 + 1) * EW * SZ : none;
    o3[6] = a3 > 0 ? self - dd - (sa + 1) * EW * SZ : none;
#pragma unroll
    for (int k = 0; k < 7; ++k) o3p[s][k] = o3[k];  // self, up e1..e3, dn e1..e3
  }
  int o2[5];
#pragma unroll
  for (int t = 0; t < S2; ++t) {
    const int p = pb2[t];
    const int b1 = p & 255, b2 = (p >> 8) & 255, tb = p >> 16;
    const int item = lane + TL * t;
    const int row = item / CH, ch = item - (item / CH) * CH;
    const int self = wb + L::cunit(row, ch) * SZ;
    o2[0] = self;
    o2[1] = wb + L::cunit(row + tb + 1, ch) * SZ;
    o2[2] = wb + L::cunit(row + tb + 2, ch) * SZ;
    o2[3] = b1 > 0 ? wb + L::cunit(row - tb, ch) * SZ : self;
    o2[4] = b2 > 0 ? wb + L::cunit(row - tb - 1, ch) * SZ : self;
#pragma unroll
    for (int k = 0; k < 5; ++k) o2p[t][k] = o2[k];  // self, up e1, e2, dn e1, e2
  }
  int lpo[S3N][4];  // lift-chain position of alpha on face f
#pragma unroll
  for (int s = 0; s < S3N; ++s) {
    const int p = pa3[s];
    const int a1 = p & 255, a2 = (p >> 8) & 255, a3 = (p >> 16) & 255, sa = p >> 24;
    const int e = (lane + TL * s) - ((lane + TL * s) / EW) * EW;
    const int af[4] = {N - sa, a1, a2, a3};
    const int b1f[4] = {a2, a2, a1, a1}, b2f[4] = {a3, a3, a3, a2};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int rem = N - af[f];  // level alpha_f of face f's chain starts at dimp(N) - dimp(N - alpha_f)
      // level base + the (swizzled) unit of the local row; zero-weighted slots use row 0
      const bool ok = af[f] >= 0;
      const int lev = ok ? NP - (rem + 1) * (rem + 2) * (rem + 3) / 6 : 0;
      lpo[s][f] = wb + (lev * CHP + L::cunit(ok ? g2(b1f[f], b2f[f]) : 0, f * EW + e)) * SZ;
    }
  }
  struct N3 {
    int self, up[3], dn[3], a1, a2, a3, sa;
  };
  auto nb3 = [&](int s) -> N3 {
    const int p = opq(pa3[s]);
    N3 r;
    r.a1 = p & 255;
    r.a2 = (p >> 8) & 255;
    r.a3 = (p >> 16) & 255;
    r.sa = p >> 24;
    r.self = o3p[s][0];
    r.up[0] = o3p[s][1];
    r.up[1] = o3p[s][2];
    r.up[2] = o3p[s][3];
    r.dn[0] = o3p[s][4];
    r.dn[1] = o3p[s][5];
    r.dn[2] = o3p[s][6];
    return r;
  };
  struct N2 {
    int self, up[2], dn[2], b1, b2, tb;
  };
  auto nb2 = [&](int t) -> N2 {
    const int p = opq(pb2[t]);
    N2 r;
    r.b1 = p & 255;
    r.b2 = (p >> 8) & 255;
    r.tb = p >> 16;
    r.self = o2p[t][0];
    r.up[0] = o2p[t][1];
    r.up[1] = o2p[t][2];
    r.dn[0] = o2p[t][3];
    r.dn[1] = o2p[t][4];
    return r;
  };

  // zero this wave's LDS slice once (stale reads are weighted by zero and must be finite)
  for (int i = lane; i < L::TOTAL; i += TL) at(wb + i * SZ) = real(0);
  if constexpr (!L::MUL_REGS) {
    for (int i = threadIdx.x; i < PTAB; i += blockDim.x) {
      const int b = i / (EW * NH), item = i - b * (EW * NH), pos = item / EW;
      int a1, a2, a3, b1, b2, b3;
      pos3(pos, a1, a2, a3);
      pos3(b, b1, b2, b3);
      const int a0 = N + M - a1 - a2 - a3, b0 = M - b1 - b2 - b3;
      const bool ok = a1 >= b1 && a2 >= b2 && a3 >= b3 && a0 >= b0;
      ptab[i] = (uint8_t)(ok ? g3(a1 - b1, a2 - b2, a3 - b3) : NP);
    }
    __syncthreads();
  }
  team_sync();

  // ---- prefetch of the next element group ------------------------------------------------
  real qn[4][S3N], pn[SPW];
  int cn[SF];
  // Every load below is unconditional: lanes without an item read a valid stand-in address
  // (element k0, which exists) and their value is discarded or replaced where it is used.
  // Loads under divergent control flow would make later writes to the same registers wait
  // for all outstanding loads, which would expose the latency that the prefetch hides.
  // Scalar r of the per-element record held by this lane. With lane reads every wave of a
  // one-element team holds the whole record (scalars 0..PW-1 in its lanes 0..PW-1).
  constexpr bool SC_LANES = EW == 1 && stage_scalars<real, N>() >= 2;
  // mode 3: geometry by lane reads, c^2 by one batch of scalar loads at the product's start
  // (one wait, no lane read per coefficient and slot)
  constexpr bool C2_BATCH = EW == 1 && stage_scalars<real, N>() == 3 && M > 0;
  static_assert(!SC_LANES || L::PW <= 64, "the per-element record must fit one wavefront");
  auto sitem = [&](int r) { return SC_LANES ? (lane & 63) + 64 * r : lane + TL * r; };
  auto prefetch = [&](int64_t g) {
    const int64_t k0 = g * EW;
#pragma unroll
    for (int s = 0; s < S3N; ++s) {
      const int item = lane + TL * s;
      const int e = item - (item / EW) * EW, pos = item / EW;
      const bool ok = item < EW * NP && k0 + e < K;
      const size_t idx = ok ? (size_t)(k0 + e) * NP + pos : (size_t)k0 * NP;
#pragma unroll
      for (int f = 0; f < 4; ++f) qn[f][s] = qin[(size_t)f * K * NP + idx];
    }
#pragma unroll
    for (int r = 0; r < SPW; ++r) {
      const int i = sitem(r);
      const int j = i - 25 * EW;
      const bool geo_ok = i < 25 * EW && k0 + i / 25 < K;
      const bool c2_ok = i >= 25 * EW && i < PW * EW && k0 + j / MP < K;
      const real* src = geo_ok ? a.geo + k0 * kGeoStride + i : (c2_ok ? a.c2 + k0 * MP + j : a.geo + k0 * kGeoStride);
      pn[r] = *src;
    }
  };
  // face connectivity of group g (4 k' + f' or -1 per flux slot)
  auto load_conn = [&](int64_t g, int (&c)[SF]) {
    const int64_t k0 = g * EW;
#pragma unroll
    for (int u = 0; u < SF; ++u) {
      const int item = lane + TL * u;
      const int fe = ffe[u] & 0xFFFF, f = fe / EW, e = fe - (fe / EW) * EW;
      const bool ok = item < 4 * EW * NFP && k0 + e < K;
      c[u] = a.conn[ok ? (k0 + e) * 4 + f : k0 * 4];  // a valid id or -1 either way
    }
  };
  // the position in qin of flux slot u's neighbour coefficient for connectivity c (boundary
  // faces, c < 0, take the group's first coefficient; the value is not used)
  auto nb_base = [&](int64_t k0, int u, int c) -> size_t {
    return c >= 0 ? (size_t)(c >> 2) * NP + ((fnb[u] >> (8 * (c & 3))) & 255) : (size_t)k0 * NP;
  };
  // one-wave teams: group g's neighbour traces straight into LDS (rows of the last slot only
  // as wide as its items)
  auto nb_dma = [&](int64_t g, const int (&c)[SF]) {
    if constexpr (L::RS_DMA) {
      const int64_t k0 = g * EW;
      const size_t fs = (size_t)K * NP;
#pragma unroll
      for (int u = 0; u < SF; ++u) {
        const size_t base = nb_base(k0, u, c[u]);
        if (u < SF - 1 || lane < L::NBLAST) {
#pragma unroll
          for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int h = 0; h < NH2; ++h) dma(nbt, (f * NH2 + h) * L::NBR + u * TL, qin + base + f * fs, h);
        }
      }
    }
  };

  // Stage group gg's scalars and state (prefetched into qn, pn) into the team's LDS slice. A
  // lane keeps the value it writes at its own position when the next phase reads that
  // position again ("self" terms below): coefficient positions are the same at every degree,
  // so the value is already in the lane's registers (qcur).
  real qcur[4][S3N], pcur[SPW];
  auto stage_group = [&](int64_t gg) {
    const int64_t kk = gg * EW;
#pragma unroll
    for (int r = 0; r < SPW; ++r) {
      const int i = sitem(r);
      const bool ok = i < 25 * EW ? kk + i / 25 < K : kk + (i - 25 * EW) / MP < K;
      pcur[r] = ok ? pn[r] : real(0);
      if (i < PW * EW && (!SC_LANES || lane < 64)) at(wb + BP + i * SZ) = pcur[r];
    }
#pragma unroll
    for (int s = 0; s < S3N; ++s) {
      const int item = lane + TL * s;
      const bool ok = kk + (item - (item / EW) * EW) < K;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        qcur[f][s] = ok ? qn[f][s] : real(0);
        if (item < EW * NP) at(wb + BQ + f * PQ + item * SZ) = qcur[f][s];
      }
    }
  };

  int64_t g = gbeg + lw;
  int cur_cn[SF];  // connectivity of the group being computed (one-wave teams; cn: the next one)
  if (g < gend) {
    prefetch(g);
    stage_group(g);
    load_conn(g, cn);
    if constexpr (L::RS_DMA) {
      nb_dma(g, cn);
#pragma unroll
      for (int u = 0; u < SF; ++u) cur_cn[u] = cn[u];
      load_conn(g + waves_per_xcd < gend ? g + waves_per_xcd : g, cn);
    }
    // wait for the connectivity here, so that the loop's first use of it does not need to
    // drain the loads and stores that the loop itself has in flight
#pragma unroll
    for (int u = 0; u < SF; ++u) asm volatile("" : "+v"(cn[u]));
  }

  for (; g < gend; g += waves_per_xcd) {
    const int64_t k0 = g * EW;
    // per-element scalars: geometry record and c^2/beta!; a one-element team reads them with
    // scalar loads (the lines were brought in by the previous iteration's prefetch), larger
    // groups from their LDS copy
    const real* const gk = a.geo + k0 * kGeoStride;
    const real* const ck = a.c2 + k0 * MP;
    auto geo_at = [&](int e, int i) -> real {
      if constexpr (SC_LANES) return lane_value(pcur[0], i);
      else if constexpr (EW == 1 && stage_scalars<real, N>() == 1) return uload(gk + i);
      else return at(wb + BP + (e * 25 + i) * SZ);
    };
    real c2s[C2_BATCH ? MP : 1];
    auto c2_at = [&](int e, int b) -> real {
      if constexpr (C2_BATCH) return c2s[b];
      else if constexpr (SC_LANES) return lane_value(pcur[0], 25 + b);
      else if constexpr (EW == 1 && stage_scalars<real, N>() == 1) return uload(ck + b);
      else return at(wb + BP + (25 * EW + e * MP + b) * SZ);
    };
    if constexpr (L::MUL_REGS) {  // keep unpacking of the product positions inside the loop
#pragma unroll
      for (int s = 0; s < S3; ++s)
#pragma unroll
        for (int b = 0; b < (MP + 1) / 2; ++b) asm volatile("" : "+v"(mpos[s][b]));
    }
    // (this group's scalars and state were staged into LDS at the end of the previous group)
    const int64_t gnext = g + waves_per_xcd;
    real nb[4][SF];
    int cur_conn[SF];
    if constexpr (L::LOADS == kLoadsEarly) {  // this group's traces, then the next group's data
#pragma unroll
      for (int u = 0; u < SF; ++u) {
        cur_conn[u] = cn[u];
        const size_t base = nb_base(k0, u, cn[u]);
        const size_t fs = (size_t)K * NP;
#pragma unroll
        for (int f = 0; f < 4; ++f) nb[f][u] = qin[base + f * fs];
      }
      // Every trace load is issued before the next group's loads, and those are issued
      // unconditionally (a stand-in group past the end), so that the flux phase can wait for
      // the traces alone: the counter of outstanding loads is in issue order, and loads on
      // one side of a branch would make the wait cover them all.
      asm volatile("" ::: "memory");
      const int64_t gn = gnext < gend ? gnext : g;
      prefetch(gn);
      load_conn(gn, cn);
    }
    team_sync();

    // ---- volume: reference derivatives at degree N-1 -----------------------------------
    // Y planes: -dp/dx, -dp/dy, -dp/dz, -div u at degree N-1 (times N/2)
    constexpr real half_n = real(N) / real(2);
    real ycar[4][S3N];
#pragma unroll
    for (int s = 0; s < S3N; ++s) ycar[0][s] = ycar[1][s] = ycar[2][s] = ycar[3][s] = real(0);
#pragma unroll
    for (int s = 0; s < S3; ++s) {
      const int item = lane + TL * s;
      if (s * TL < EW * NP1 && item < EW * NP1) {
        const int e = item - (item / EW) * EW;
        const N3 x = nb3(s);
        const int self = x.self;
        real v0[4], v1[4], v2[4], v3[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          v0[f] = (BBW_CARRY & 1) ? qcur[f][s < S3N ? s : 0] : at(self + BQ + f * PQ);
          v1[f] = at(x.up[0] + BQ + f * PQ);
          v2[f] = at(x.up[1] + BQ + f * PQ);
          v3[f] = at(x.up[2] + BQ + f * PQ);
        }
        real dv = 0;
        real gr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const real G0 = geo_at(e, 3 * i), G1 = geo_at(e, 3 * i + 1), G2 = geo_at(e, 3 * i + 2);
          gr[i] = -half_n * (G0 * (v1[0] - v0[0]) + G1 * (v2[0] - v0[0]) + G2 * (v3[0] - v0[0]));
          dv += G0 * (v1[1 + i] - v0[1 + i]) + G1 * (v2[1 + i] - v0[1 + i]) + G2 * (v3[1 + i] - v0[1 + i]);
        }
        const int sn = s < S3N ? s : 0;
        ycar[0][sn] = gr[0];
        ycar[1][sn] = gr[1];
        ycar[2][sn] = gr[2];
        ycar[3][sn] = -half_n * dv;
#pragma unroll
        for (int c = 0; c < 4; ++c) at(self + BA + c * PY) = ycar[c][sn];
      }
    }
    team_sync();
    // elevate to degree N: acc[0] = -div u, acc[1 + i] = -d p / d x_i
    real acc[4][S3N] = {};
    constexpr real inv_n = real(1) / real(N);
#pragma unroll
    for (int s = 0; s < S3N; ++s) {
      const int item = lane + TL * s;
      if (item >= EW * NP) continue;
      const N3 x = nb3(s);
      const int self = x.self;
      const real w0 = real(N - x.sa) * inv_n, w1 = real(x.a1) * inv_n, w2 = real(x.a2) * inv_n,
                 w3 = real(x.a3) * inv_n;
      real t[4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        t[c] = w0 * ((BBW_CARRY & 2) ? ycar[c][s] : at(self + BA + c * PY)) + w1 * at(x.dn[0] + BA + c * PY) + w2 * at(x.dn[1] + BA + c * PY) +
               w3 * at(x.dn[2] + BA + c * PY);
      acc[0][s] = t[3];
      acc[1][s] = t[0];
      acc[2][s] = t[1];
      acc[3][s] = t[2];
    }
    team_sync();

    // ---- surface: penalty fluxes per face coefficient ------------------------------------
    // F [NFP*CHP] at BA, channel (type*4 + f)*EW + e; T [NFP1*CHP] right after it
    constexpr int BF = BA, BT = BA + CHP * NFP * SZ;
    // the neighbour traces of this group: in registers since the top, in LDS since the previous
    // group, or requested here so that their registers are not held through the volume phases
#pragma unroll
    for (int u = 0; u < SF; ++u) {
      if constexpr (L::LOADS == kLoadsLds) {
        cur_conn[u] = cur_cn[u];
      } else if constexpr (L::LOADS == kLoadsLate) {
        const int c = cn[u];
        cur_conn[u] = c;
        const size_t base = nb_base(k0, u, c);
        const size_t fs = (size_t)K * NP;
#pragma unroll
        for (int f = 0; f < 4; ++f) nb[f][u] = qin[base + f * fs];
      }
    }
#pragma unroll
    for (int u = 0; u < SF; ++u) {
      const int item = lane + TL * u;
      if (item < 4 * EW * NFP) {
        const int fe = ffe[u] & 0xFFFF, m = ffe[u] >> 16;
        const int f = fe / EW, e = fe - (fe / EW) * EW;
        const real pm = at(fown[u] + BQ), um = at(fown[u] + BQ + PQ), vm = at(fown[u] + BQ + 2 * PQ),
                   wm = at(fown[u] + BQ + 3 * PQ);
        const int gf = wb + BP + (e * 25 + 9 + 4 * f) * SZ;
        const real nx = at(gf + SZ), ny = at(gf + 2 * SZ), nz = at(gf + 3 * SZ);
        // jumps [[p]] = p+ - p and [[u]].n against the neighbour, or against the mirror
        // state on a wall: p = 0 walls take p+ = -p, u+ = u; rigid walls p+ = p,
        // u+ = u - 2 (u.n) n, so [[u]].n = -2 u.n (unit normals)
        real nbv[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          if constexpr (L::RS_DMA) nbv[f] = lds_real(nbt, f * NH2 * L::NBR + u * TL, L::NBR);
          else nbv[f] = nb[f][u];
        }
        const real jp_in = nbv[0] - pm;
        const real jun_in = (nbv[1] - um) * nx + (nbv[2] - vm) * ny + (nbv[3] - wm) * nz;
        const real jp_wall = a.bc == 0 ? real(-2) * pm : real(0);
        const real jun_wall = a.bc == 0 ? real(0) : real(-2) * (um * nx + vm * ny + wm * nz);
        const bool interior = cur_conn[u] >= 0;
        const real jp = interior ? jp_in : jp_wall;
        const real jun = interior ? jun_in : jun_wall;
        at(wb + BF + L::cunit(m, fe) * SZ) = real(0.5) * (a.tau_p * jp - jun);
        at(wb + BF + L::cunit(m, fe + 4 * EW) * SZ) = real(0.5) * (a.tau_u * jun - jp);
      }
    }
    // the RK register of this group (straight into LDS, read by the update at the end, or
    // into registers for a multi-wave team), then the next group's state, geometry and c^2
    real rs[L::RS_DMA ? 1 : 4][L::RS_DMA ? 1 : S3N];
    if constexpr (UPDATE && !L::RS_DMA) {
#pragma unroll
      for (int s = 0; s < S3N; ++s) {
        const int item = lane + TL * s;
        const int e = item - (item / EW) * EW, pos = item / EW;
        const bool ok = item < EW * NP && k0 + e < K;
        const size_t idx = ok ? (size_t)(k0 + e) * NP + pos : (size_t)k0 * NP;  // see the prefetch
#pragma unroll
        for (int f = 0; f < 4; ++f) rs[f][s] = a.res[(size_t)f * K * NP + idx];
      }
    }
    if constexpr (UPDATE && L::RS_DMA) {
#pragma unroll
      for (int s = 0; s < S3N; ++s) {
        const int item = lane + TL * s;
        const int e = item - (item / EW) * EW, pos = item / EW;
        const bool ok = item < EW * NP && k0 + e < K;
        const size_t idx = ok ? (size_t)(k0 + e) * NP + pos : (size_t)k0 * NP;  // see the prefetch
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
          for (int h = 0; h < NH2; ++h) dma(rbt, ((f * S3N + s) * NH2 + h) * TL, a.res + (size_t)f * K * NP + idx, h);
      }
    }
    if constexpr (L::LOADS == kLoadsLds) {
      // unconditional, with a stand-in group past the end (values unused): a load under a
      // branch would make its registers' next readers wait for every outstanding load
      const int64_t gn = gnext < gend ? gnext : g, gnn = gnext + waves_per_xcd < gend ? gnext + waves_per_xcd : g;
      nb_dma(gn, cn);  // cn holds the next group's connectivity
#pragma unroll
      for (int u = 0; u < SF; ++u) cur_cn[u] = cn[u];
      prefetch(gn);
      load_conn(gnn, cn);
    } else if (L::LOADS == kLoadsLate) {
      const int64_t gn = gnext < gend ? gnext : g;  // unconditional, as above
      prefetch(gn);
      load_conn(gn, cn);
    }
    team_sync();

    // ---- lift: L_0 on each face flux, then the layer chain (levels pre-scaled by l_i) -----
    real ccar[S2];  // the lane's own face-chain value of the previous lift phase
#pragma unroll
    for (int t = 0; t < S2; ++t) ccar[t] = real(0);
#pragma unroll
    for (int t = 0; t < S2; ++t) {  // T = (E^N_{N-1})^T F
      const int item = lane + TL * t;
      if (t * TL < CH * NFP1 && item < CH * NFP1) {
        const N2 x = nb2(t);
        ccar[t] = inv_n * (real(N - x.tb) * at(x.self + BF) + real(x.b1 + 1) * at(x.up[0] + BF) +
                           real(x.b2 + 1) * at(x.up[1] + BF));
        at(x.self + BT) = ccar[t];
      }
    }
    team_sync();
    constexpr int BC = BB;  // chain [NP*CHP], level i at chain_off(N, i)*CHP
    {
      constexpr real l0a = real(2 * N + 3) / real(2);
      constexpr real l0b = real(N * N) / real(2) / real(N);
#pragma unroll
      for (int t = 0; t < S2; ++t) {  // level 0 = L_0 F = (2N+3)/2 F + N^2/2 E T
        const int item = lane + TL * t;
        if (item < CH * NFP) {
          const N2 x = nb2(t);
          const real et = real(N - x.tb) * ((BBW_CARRY & 4) ? ccar[t] : at(x.self + BT)) + real(x.b1) * at(x.dn[0] + BT) + real(x.b2) * at(x.dn[1] + BT);
          ccar[t] = l0a * at(x.self + BF) + l0b * et;
          at(x.self + BC) = ccar[t];
        }
      }
    }
    team_sync();
#pragma unroll
    for (int i = 1; i <= N; ++i) {
      const int n = N - i + 1;  // level i-1 has degree n
      const real sc = real(lift_ell(N, i) / lift_ell(N, i - 1)) / real(n);
      const int cnt = CH * dim2(n - 1);
      const int src = BC + chain_off(N, i - 1) * CHP * SZ, dst = BC + chain_off(N, i) * CHP * SZ;
#pragma unroll
      for (int t = 0; t < S2; ++t) {
        const int item = lane + TL * t;
        if (t * TL < cnt && item < cnt) {
          const N2 x = nb2(t);
          ccar[t] = sc * (real(n - x.tb) * ((BBW_CARRY & 4) ? ccar[t] : at(x.self + src)) + real(x.b1 + 1) * at(x.up[0] + src) +
                          real(x.b2 + 1) * at(x.up[1] + src));
          at(x.self + dst) = ccar[t];
        }
      }
      team_sync();
    }
    // gather the four face lifts into every coefficient (and add the projected source to r_p)
    constexpr int BR = BA;  // r_p / alpha! (degree N); F and T are dead once level 0 is formed
#pragma unroll
    for (int s = 0; s < S3N; ++s) {
      const int item = lane + TL * s;
      if (item < EW * NP) {
        const int e = item - (item / EW) * EW;
        if (a.src) {  // the projected pressure source s(t) g (a uniform branch; no registers held otherwise)
          const size_t idx = k0 + e < K ? (size_t)(k0 + e) * NP + item / EW : (size_t)k0 * NP;
          acc[0][s] += a.src_amp * a.src[idx];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const int lpf = lpo[s][f];
          const real sc = geo_at(e, 9 + 4 * f);
          const real lpv = at(lpf + BC);
          // the u channel (channel + 4 EW) of the same row: with a swizzle and 4 EW < 8 it
          // is the slot with bit 2 flipped (rows are 8-real aligned), else a fixed offset
          constexpr bool flip = L::SWZ && (4 * EW) % 8 != 0;
          const int lpu = flip ? ((lpf + BC) ^ (4 * SZ)) : (lpf + BC + 4 * EW * SZ);
          const real luv = at(lpu) * sc;
          acc[0][s] += sc * lpv;
          acc[1][s] += geo_at(e, 10 + 4 * f) * luv;
          acc[2][s] += geo_at(e, 11 + 4 * f) * luv;
          acc[3][s] += geo_at(e, 12 + 4 * f) * luv;
        }
        if constexpr (RPOUT)  // r_p before the weight adjustment (a separate instance, step mode)
          if (k0 + e < K) a.rp_out[(size_t)(k0 + e) * NP + item / EW] = acc[0][s];
        if constexpr (M > 0) {
          at(wb + BR + item * SZ) = acc[0][s] * fac3[s];
          if constexpr (!L::MUL_REGS)
            if (s == 0 && lane < EW) at(wb + BR + (NP * EW + lane) * SZ) = real(0);  // the zero cell
        } else {
          acc[0][s] *= c2_at(e, 0);
        }
      }
    }

    // ---- WADG: product with c^2_M, M reductions, telescoped projection -----------------
    if constexpr (M > 0) {
      team_sync();
      constexpr int NH1 = L::NH1;
      constexpr int BH = BB, BH1 = BB + EW * NH * SZ, BL = BH1 + EW * NH1 * SZ;
      // FP64 levels: item u of a level at byte BLD + (level offset + u) * 8; a 3D offset
      // o = wb + 4 u (float slots) maps to wb + 8 u by 2 o - wb
      constexpr int BLD = (BL + 7) & ~7;
      auto atd = [lds](int byteoff) -> double& { return *reinterpret_cast<double*>(lds + byteoff); };
      auto dof = [wb](int off) { return 2 * off - wb; };
      real wcar[S3];  // the lane's own value of the previous WADG phase
#pragma unroll
      for (int s = 0; s < S3; ++s) wcar[s] = real(0);
      // re-zero the guards in front of levels 1..N (the face chain shared this space)
      if (lane < N * EW) {
        if constexpr (L::TELE64) atd(wb + BLD + ((lev_off(N, lane / EW + 1) - 1) * EW + lane % EW) * 8) = 0.0;
        else at(wb + BL + ((lev_off(N, lane / EW + 1) - 1) * EW + lane % EW) * SZ) = real(0);
      }
      // h_gamma = sum_beta R_{gamma-beta} c2_beta/beta!
      if constexpr (C2_BATCH) {
#pragma unroll
        for (int b = 0; b < MP; ++b) c2s[b] = uload(ck + b);
      }
      real h[S3];
#pragma unroll
      for (int s = 0; s < S3; ++s) h[s] = real(0);
      if constexpr (L::MUL_REGS) {  // few terms: positions in registers, slot by slot
#pragma unroll
        for (int s = 0; s < S3; ++s) {
          const int item = lane + TL * s;
          if (item < EW * NH) {
            const int e = item - (item / EW) * EW;
#pragma unroll
            for (int b = 0; b < MP; ++b) {
              const int off = (b % 2 == 0) ? (mpos[s][b / 2] & 0xFFFF) : ((unsigned)mpos[s][b / 2] >> 16);
              h[s] += at(off) * c2_at(e, b);
            }
          }
        }
      } else {  // many terms: positions from the table, slot by slot. A full slot has no
                // branch and the partial last slot one branch around all of its terms, so
                // that the table and value reads of consecutive terms can be in flight
                // together (a branch per term would wait for each term's reads in turn).
        auto slot_terms = [&](int s) {
          const int item = lane + TL * s, e = item - (item / EW) * EW;
#pragma unroll
          for (int b = 0; b < MP; ++b) {
            const int off = wb + BR + ((int)ptab[b * (EW * NH) + item] * EW + e) * SZ;
            h[s] += at(off) * c2_at(e, b);
            // close a batch: its sum is formed before the next batch's reads are issued
            constexpr int PB = stage_batch<real, N>();
            if (b % PB == PB - 1) asm volatile("" : "+v"(h[s])::"memory");
          }
        };
#pragma unroll
        for (int s = 0; s < S3; ++s) {
          if ((s + 1) * TL <= EW * NH) slot_terms(s);
          else if (lane + TL * s < EW * NH) slot_terms(s);
        }
      }
#pragma unroll
      for (int s = 0; s < S3; ++s) {
        const int item = lane + TL * s;
        if (item < EW * NH) {
          wcar[s] = h[s] * facH[s];
          at(wb + BH + item * SZ) = wcar[s];
        }
      }
      team_sync();
      // M reductions: degree N+M -> N; the last one writes level 0 of the telescoping
#pragma unroll
      for (int n = N + M; n > N; --n) {
        const int src = ((N + M - n) % 2 == 0) ? BH : BH1;
        const int dst = (n - 1 == N) ? BL : (((N + M - n) % 2 == 0) ? BH1 : BH);
        const real inv = real(1) / real(n);
        const int cnt = EW * dimp(n - 1);
#pragma unroll
        for (int s = 0; s < S3; ++s) {
          const int item = lane + TL * s;
          if (s * TL < cnt && item < cnt) {
            const N3 x = nb3(s);
            const real self_v = (BBW_CARRY & 8) ? wcar[s] : at(x.self + src);
            wcar[s] = inv * (real(n - x.sa) * self_v + (at(x.up[0] + src) + at(x.up[1] + src) + at(x.up[2] + src)));
            if (L::TELE64 && n - 1 == N) atd(dof(x.self) + BLD) = double(wcar[s]);
            else at(x.self + dst) = wcar[s];
          }
        }
        team_sync();
      }
      if constexpr (L::TELE64) {
        // FP32 state, FP64 telescoping. The c_j alternate in sign and grow with N (sum |c_j|
        // = 259 at N=8, M=4 and 524 at N=9, M=4), so float sweeps lose about that factor of
        // their precision. Here the sweeps of the FP64 kernel run on doubles in LDS: level 0
        // (the float reductions' output) is widened once and the result rounded to float.
        double wd[S3N];
#pragma unroll
        for (int s = 0; s < S3N; ++s) wd[s] = double(wcar[s]);
#pragma unroll
        for (int j = 1; j <= N; ++j) {
          const int n = N - j + 1;
          const double inv = 1.0 / double(n);
          const int cnt = EW * dimp(n - 1);
          const int src = BLD + lev_off(N, j - 1) * EW * 8, dst = BLD + lev_off(N, j) * EW * 8;
#pragma unroll
          for (int s = 0; s < S3N; ++s) {
            const int item = lane + TL * s;
            if (s * TL < cnt && item < cnt) {
              const N3 x = nb3(s);
              wd[s] = inv * (double(n - x.sa) * wd[s] +
                             (atd(dof(x.up[0]) + src) + atd(dof(x.up[1]) + src) + atd(dof(x.up[2]) + src)));
              atd(dof(x.self) + dst) = wd[s];
            }
          }
          team_sync();
        }
        if (lane < EW) {
          wd[0] *= a.cjd[N];
          atd(wb + BLD + (lev_off(N, N) * EW + lane) * 8) = wd[0];
        }
        team_sync();
#pragma unroll
        for (int j = N - 1; j >= 0; --j) {
          const int n = N - j;
          const double inv = 1.0 / double(n);
          const double cj = a.cjd[j];
          const int cnt = EW * dimp(n);
          const int lo = BLD + lev_off(N, j) * EW * 8, hi = BLD + lev_off(N, j + 1) * EW * 8;
#pragma unroll
          for (int s = 0; s < S3N; ++s) {
            const int item = lane + TL * s;
            if (s * TL < cnt && item < cnt) {
              const N3 x = nb3(s);
              const double el = double(n - x.sa) * wd[s] +
                                (atd(dof(x.dn[0]) + hi) + atd(dof(x.dn[1]) + hi) + atd(dof(x.dn[2]) + hi));
              wd[s] = (cj * iA2d[s]) * atd(dof(x.self) + lo) + inv * el;
              atd(dof(x.self) + lo) = wd[s];
            }
          }
          team_sync();
        }
#pragma unroll
        for (int s = 0; s < S3N; ++s) {
          const int item = lane + TL * s;
          if (item < EW * NP) acc[0][s] = real(double(aF[s]) * wd[s]);
        }
      } else {
        // downward sweep: level j = (E^{N-j+1}_{N-j})^T level j-1
#pragma unroll
        for (int j = 1; j <= N; ++j) {
          const int n = N - j + 1;
          const real inv = real(1) / real(n);
          const int cnt = EW * dimp(n - 1);
          const int src = BL + lev_off(N, j - 1) * EW * SZ, dst = BL + lev_off(N, j) * EW * SZ;
#pragma unroll
          for (int s = 0; s < S3N; ++s) {
            const int item = lane + TL * s;
            if (s * TL < cnt && item < cnt) {
              const N3 x = nb3(s);
              const real self_v = (BBW_CARRY & 8) ? wcar[s] : at(x.self + src);
              wcar[s] = inv * (real(n - x.sa) * self_v + (at(x.up[0] + src) + at(x.up[1] + src) + at(x.up[2] + src)));
              at(x.self + dst) = wcar[s];
            }
          }
          team_sync();
        }
        // upward sweep: s_N = c_N r_N; s_j = c_j r_j + E^{N-j}_{N-j-1} s_{j+1}. The
        // reductions above kept A(alpha) x (one weight, n - |a|, on the e0 term); here s is
        // kept as s / A(alpha), so r enters with 1/A^2 and the elevation again has one weight.
        if (lane < EW) {
          wcar[0] *= a.cj[N];
          at(wb + BL + (lev_off(N, N) * EW + lane) * SZ) = wcar[0];
        }
        team_sync();
#pragma unroll
        for (int j = N - 1; j >= 0; --j) {
          const int n = N - j;
          const real inv = real(1) / real(n);
          const real cj = a.cj[j];
          const int cnt = EW * dimp(n);
          const int lo = BL + lev_off(N, j) * EW * SZ, hi = BL + lev_off(N, j + 1) * EW * SZ;
#pragma unroll
          for (int s = 0; s < S3N; ++s) {
            const int item = lane + TL * s;
            if (s * TL < cnt && item < cnt) {
              const N3 x = nb3(s);
              const real self_v = (BBW_CARRY & 8) ? wcar[s] : at(x.self + hi);
              const real el = real(n - x.sa) * self_v + (at(x.dn[0] + hi) + at(x.dn[1] + hi) + at(x.dn[2] + hi));
              wcar[s] = (cj * iA2[s]) * at(x.self + lo) + inv * el;
              at(x.self + lo) = wcar[s];
            }
          }
          team_sync();
        }
#pragma unroll
        for (int s = 0; s < S3N; ++s) {
          const int item = lane + TL * s;
          if (item < EW * NP) acc[0][s] = aF[s] * wcar[s];
        }
      }
    }

    // ---- write: rhs, or the low-storage RK stage --------------------------------------------
    // The results are formed first; the next group is then staged into LDS (its loads have
    // arrived), and only then are the results stored, so the next group's first reads of its
    // own data never have to wait for these stores.
    real outv[4][S3N], resv[4][S3N];
#pragma unroll
    for (int s = 0; s < S3N; ++s) {
      const int item = lane + TL * s;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if constexpr (UPDATE) {
          real rv;
          if constexpr (L::RS_DMA) rv = lds_real(rbt, ((f * S3N + s) * NH2) * TL, TL);
          else rv = rs[f][s];
          resv[f][s] = a.rk_a * rv + a.dt * acc[f][s];
          outv[f][s] = at(wb + BQ + f * PQ + (item < EW * NP ? item : 0) * SZ) + a.rk_b * resv[f][s];
        } else {
          outv[f][s] = acc[f][s];
        }
      }
    }
    team_sync();  // the next group overwrites this team's LDS slice
    stage_group(gnext < gend ? gnext : g);  // a stand-in past the end (unused)
#pragma unroll
    for (int s = 0; s < S3N; ++s) {
      const int item = lane + TL * s;
      const int e = item - (item / EW) * EW, pos = item / EW;
      if (item < EW * NP && k0 + e < K) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const size_t gi = ((size_t)f * K + k0 + e) * NP + pos;
          if constexpr (UPDATE) a.res[gi] = resv[f][s];
          a.qout[gi] = outv[f][s];
        }
      }
    }
  }
}

template <typename real, int N, int M, bool UPDATE, bool RPOUT = false>
int launch_stage_typed(const StageArgs<real>& a, void* stream) {
  constexpr int EW = elems_per_wave<N>();
  using L = StageLayout<real, N, M, EW>;
  constexpr int WPB = L::WPB;
  auto kern = stage_kernel<real, N, M, EW, WPB, UPDATE, RPOUT>;
  // persistent grid: the blocks resident on the current device, a multiple of 8; computed
  // once per device (benign if two threads compute it concurrently: same value)
  constexpr int kMaxDevices = 64;
  static std::atomic<int> grids[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return (int)hipErrorInvalidDevice;
  int grid = dev < kMaxDevices ? grids[dev].load(std::memory_order_relaxed) : 0;
  if (grid == 0) {
    int ncu = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 256;
    int per_cu = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WPB, 0);
    if (getenv("BBWADG_DEBUG")) {
      hipFuncAttributes attr{};
      (void)hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kern));
      fprintf(stderr, "bbwadg: N=%d M=%d sizeof(real)=%d WPB=%d occupancy blocks/CU=%d numRegs=%d lds=%zu\n", N, M,
              (int)sizeof(real), WPB, per_cu, attr.numRegs, (size_t)attr.sharedSizeBytes);
    }
    const char* env = getenv("BBWADG_BLOCKS_PER_CU");  // tuning override
    if (env && *env) per_cu = atoi(env);
    if (per_cu <= 0) per_cu = 1;
    grid = ncu * per_cu;
    grid = (grid / 8) * 8 > 0 ? (grid / 8) * 8 : grid;
    if (dev < kMaxDevices) grids[dev].store(grid, std::memory_order_relaxed);
  }
  const int64_t groups = (a.K + EW - 1) / EW;
  const int64_t need = (groups + L::TPB - 1) / L::TPB;  // one team per element group
  int blocks = grid;
  if (need < blocks) blocks = (int)(need >= 8 ? (need / 8) * 8 : need);
  if (blocks <= 0) return 0;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * WPB), 0, (hipStream_t)stream, a);
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

template <int N, int M>
int dispatch_nm(bool update, bool f64, const void* args, void* stream) {
  if (f64) {
    const auto& a = *static_cast<const StageArgs<double>*>(args);
    if (!update) return launch_stage_typed<double, N, M, false>(a, stream);
    return a.rp_out ? launch_stage_typed<double, N, M, true, true>(a, stream) : launch_stage_typed<double, N, M, true>(a, stream);
  }
  const auto& a = *static_cast<const StageArgs<float>*>(args);
  if (!update) return launch_stage_typed<float, N, M, false>(a, stream);
  return a.rp_out ? launch_stage_typed<float, N, M, true, true>(a, stream) : launch_stage_typed<float, N, M, true>(a, stream);
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
