// Internal declarations shared by the host side of the library and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bbw {

constexpr int kMaxN = 9;
constexpr int kMaxM = 4;
constexpr int kMaxDeg = kMaxN + kMaxM;
constexpr uint16_t kNone = 0xFFFF;

// Number of Bernstein coefficients of degree n on a tetrahedron / triangle.
__host__ __device__ constexpr int dimp(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) * (n + 3) / 6; }
__host__ __device__ constexpr int dim2(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) / 2; }

// Offsets (in uint16 entries) of the index tables inside one device buffer. Entries are
// groups of 4 uint16; unused slots hold kNone.
//   mi3[n]  : [dimp(n)][4]    multi-index (a0..a3) of each degree-n coefficient
//   el3[n]  : [dimp(n)][4]    index at degree n-1 of gamma - e_k (kNone if gamma_k = 0)
//   red3[n] : [dimp(n-1)][4]  index at degree n of alpha + e_k
//   mi2[n]  : [dim2(n)][4]    face multi-index (b0,b1,b2,-)
//   el2     : [dim2(N)][4]    face index at degree N-1 of gamma - e_k (kNone if 0)
//   red2[n] : [dim2(n-1)][4]  face index at degree n of beta + e_k (slot 3 unused)
//   fidx    : [4][dim2(N)]    volume index of face coefficient m of face f (one uint16 each)
//   liftpos : [4][dimp(N)]    position of alpha in face f's lift chain (one uint16 each)
//   mulidx  : [dimp(N+M)][dimp(M)]  index at degree N of gamma - beta, or kNone
struct TableOffsets {
  int32_t mi3[kMaxDeg + 1];
  int32_t el3[kMaxDeg + 1];
  int32_t red3[kMaxDeg + 1];
  int32_t mi2[kMaxN + 1];
  int32_t el2;
  int32_t red2[kMaxN + 1];
  int32_t fidx;
  int32_t liftpos;
  int32_t mulidx;
  int32_t total;
};

// Per-element geometry record: G[9] (G[3i+j] = d r_j / d x_i), then for each face f:
// Fscale_f, n_f (3 values).
constexpr int kGeoStride = 25;

template <typename real>
struct StageArgs {
  const real* qin;        // [4][K][Np] state read (own coefficients and neighbour traces)
  real* qout;             // [4][K][Np] next state (step) or rhs (rhs mode)
  real* res;              // [4][K][Np] 2N-storage register (step mode)
  const real* geo;        // [K][kGeoStride]
  const int32_t* conn;    // [K][4]: 4*k'+f' or -1 (boundary)
  const real* c2;         // [K][Mp]
  const uint16_t* tab;    // index tables
  const real* mulw;       // [dimp(N+M)][dimp(M)] multiplication weights
  TableOffsets off;
  int64_t K;
  real tau_p, tau_u;
  int32_t bc;             // 0: p = 0 walls, 1: rigid walls
  real rk_a, rk_b, dt;    // stage coefficients (step mode)
  real cj[kMaxN + 1];     // telescoped projection coefficients c_j
  real ell[kMaxN + 1];    // lift layer factors l_i
};

// Launch one fused stage (UPDATE) or one right-hand-side evaluation on `stream`.
// Returns a hipError_t value cast to int.
int launch_stage_f64(int N, int M, bool update, const StageArgs<double>& a, void* stream);
int launch_stage_f32(int N, int M, bool update, const StageArgs<float>& a, void* stream);

// Per-field squared L^2 norms in FP64 (mass matrix closed form); writes partial sums
// [nblocks][4] into `partial` (device), returns the hip error code.
int launch_l2norm(int N, int dtype, const void* q, int64_t K, const double* J, const double* mass,
                  double* partial, int nblocks, void* stream);

}  // namespace bbw
