// Internal declarations shared by the host side of the library and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bbw {

constexpr int kMaxN = 9;
constexpr int kMaxM = 4;
constexpr int kMaxDeg = kMaxN + kMaxM;

// Number of Bernstein coefficients of degree n on a tetrahedron / triangle.
__host__ __device__ constexpr int dimp(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) * (n + 3) / 6; }
__host__ __device__ constexpr int dim2(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) / 2; }

// Smallest degree whose FP32 kernels run the telescoped projection in FP64.
#ifndef BBW_TELE64_MIN_N
#define BBW_TELE64_MIN_N 8
#endif

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
  const real* c2;         // [K][Mp] c^2_M coefficients divided by beta!
  int64_t K;
  real tau_p, tau_u;
  int32_t bc;             // 0: p = 0 walls, 1: rigid walls
  real rk_a, rk_b, dt;    // stage coefficients (step mode)
  const real* src;        // [K][Np] pressure source g (coefficients), or null
  real src_amp;           // s(t) of the source f = s(t) g(x) at this stage's time
  real* rp_out;           // [K][Np] r_p before the weight adjustment (source included), or null (step mode)
  real cj[kMaxN + 1];     // telescoped projection coefficients c_j
  double cjd[kMaxN + 1];  // the c_j in FP64 (FP32 kernels that run the telescoping in FP64)
};

// Launch one fused stage (UPDATE) or one right-hand-side evaluation on `stream`.
// Returns a hipError_t value cast to int.
int launch_stage_f64(int N, int M, bool update, const StageArgs<double>& a, void* stream);
int launch_stage_f32(int N, int M, bool update, const StageArgs<float>& a, void* stream);

// Per-field squared L^2 norms in FP64 (mass matrix closed form); writes partial sums
// [nblocks][4] into `partial` (device), returns the hip error code.
int launch_l2norm(int N, int dtype, const void* q, int64_t K, const double* J, const double* mass,
                  double* partial, int nblocks, void* stream);

// The norm reduction without allocation (noalloc.hip): partial sums in a fixed device array
// of kScratchBlocks x 4 doubles, added on the device into out (device double[4]).
// scratch_init() resolves the array's address on the current device (once per device);
// both return a hipError_t value cast to int.
constexpr int kScratchBlocks = 1024;
int scratch_init();
int l2norm2_noalloc(int N, int dtype, const void* q, int64_t K, const double* J, const double* mass, int nblocks,
                    double* out, void* stream);

// Quadrature reductions over elements [k0, k1): mode 0 = squared L^2 error against
// `exact`, mode 1 = the two halves of the acoustic energy (p^2/c^2 and |u_i|^2 terms).
struct QuadReduceArgs {
  const void* q;          // [4][K][Np] state, context dtype
  const void* c2;         // [K][Mp] c^2_M coefficients, context dtype (mode 1)
  const double* J;        // [K]
  const double* basis;    // [Np][nq] B^N_alpha at the rule points
  const double* basis_c2; // [Mp][nq] B^M_beta at the rule points (mode 1)
  const double* w;        // [nq] rule weights (reference volume 4/3)
  const double* exact;    // [4][k1-k0][nq] reference values (mode 0)
  double* partial;        // [nblocks][4] per-block sums
  int64_t K, k0, k1;
  int32_t Np, Mp, nq;
};
int quad_reduce_blocks(int64_t nelems, int max_blocks);

// Dense quadrature WADG update out = P_q diag(c2q) V_q r (FP64 or FP32), tables in MFMA
// operand order:
// va[qc][ks][lane] = V_q[16 qc + lane%16][4 ks + lane/16] (NQP/16 x NPP/4 x 64) and
// pa[qc][t][ks][lane] = P_q[16 t + lane%16][16 qc + 4 ks + lane/16] (NQP/16 x NPP/16 x 4 x 64),
// zero-padded to NPP = 16 ceil(Np/16) and NQP = 16 ceil(Nq/16).
template <typename real>
struct DenseArgs {
  const real* r;    // [K][Np] input coefficients
  real* out;        // [K][Np] result (may alias r: each tile stages its inputs first)
  const real* va;
  const real* pa;
  const real* c2q;  // [K][nqp] c^2 at the points (padding zero)
  int64_t K;
  int32_t nqc;      // NQP / 16
  int32_t nqp;      // NQP
};
template <typename real>
int launch_wadg_dense(int N, const DenseArgs<real>& a, void* stream);

// Weight-adjusted update of the 9 elastic fields (elastic_kernel.hip): r, out [9][K][Np]
// (v1, v2, v3, sigma xx, yy, zz, yz, xz, xy); weights [K][Mp] as Bernstein coefficients.
template <typename real>
struct ElasticArgs {
  const real* r;
  real* out;
  const real* rho_inv;
  const real* lam;
  const real* mu;
  int64_t K;
  real cj[kMaxN + 1];
  double cjd[kMaxN + 1];  // as in StageArgs
  // optional low-storage RK stage in place of out (res != nullptr): res = rk_a res + dt u,
  // q += rk_b res, u the update of r; res, q [9][K][Np]
  real* res;
  real* q;
  real rk_a, rk_b, dt;
};
template <typename real>
int launch_elastic_update(int N, int M, const ElasticArgs<real>& a, void* stream);
// The same kernel on one field with one weight (rho_inv holds the weight, r/out [K][Np]):
// out = Pi_N(w r), the acoustic weight-adjusted update on its own.
template <typename real>
int launch_wadg_update(int N, int M, const ElasticArgs<real>& a, void* stream);

// DG right-hand side of the elastic system before the weight adjustment
// (elastic_rhs_kernel.hip): q, out [9][K][Np].
template <typename real>
struct ElasticRhsArgs {
  const real* q;
  real* out;
  const real* geo;       // [K][kGeoStride]
  const int32_t* conn;   // [K][4]
  const int32_t* fpos;   // [4][Nfp] volume position of face coefficient m of face f
  int64_t K;
  real tau_v, tau_s;
  int32_t wall;          // 0: traction-free, 1: rigid
};
template <typename real>
int launch_elastic_rhs(int N, const ElasticRhsArgs<real>& a, void* stream);

// Adjoint helpers (adjoint_kernel.hip); each returns a hipError_t value cast to int.
// Tables at the dense rule (exact to degree 2N + M), in MFMA operand order as DenseArgs:
// va = V_q (NQP/16 x NPP/4 x 64) and bwa[qc][ks][lane] = w_q B^M_g(x_q) for
// g = lane%16, q = 16 qc + 4 ks + lane/16 (zero for g >= Mp or padding points).
template <typename real>
struct C2GradArgs {
  const real* y;       // [K][Np] pressure part of the DG right-hand side of the stage input
  const real* v;       // [K][Np] pressure part of the reversed stage's adjoint variable
  const double* va;
  const double* bwa;   // [NQP/16][4][64]
  const double* J;     // [K]
  double* grad;        // [K][Mp] accumulated
  double scale;
  int64_t K;
  int32_t Mp, nqc;
};
template <typename real>
int launch_lincomb(real* x, const real* y, double alpha, double beta, int64_t n, void* stream);
template <typename real>
int launch_back_update(real* zq, real* v, const real* t, double dt, double a, double b, bool update_v, int64_t n,
                       void* stream);
template <typename real>
int launch_sample(const real* qp, const int32_t* elem, const double* basis, int32_t nrec, int32_t Np, double* out,
                  void* stream);
template <typename real>
int launch_inject(real* zp, const int32_t* elem, const double* kvec, const double* resid, int32_t nrec, int32_t Np,
                  void* stream);
template <typename real>
int launch_c2grad(int N, const C2GradArgs<real>& a, void* stream);
int launch_quad_reduce(int dtype, int mode, const QuadReduceArgs& a, int nblocks, void* stream);

}  // namespace bbw
