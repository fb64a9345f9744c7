// Host side of the BBWADG library: mesh ingest, affine geometry, face connectivity,
// Bernstein operator tables, FP64 L^2 projections, the C ABI and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <unordered_map>
#include <type_traits>
#include <vector>

#include "../../include/bbwadg.h"
#include "bbwadg_internal.hpp"

#include "surrogate_internal.hpp"

using namespace bbw;
typedef long double ld;

namespace {

thread_local std::string g_err;

int vfail(int code, const char* fmt, va_list ap) {
  char buf[512];
  vsnprintf(buf, sizeof buf, fmt, ap);
  g_err = buf;
  return code;
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vfail(code, fmt, ap);
  va_end(ap);
  return code;
}

// ------------------------------------------------------------------ combinatorics
ld factl(int n) {
  ld r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}
ld binoml(int n, int k) {
  if (k < 0 || k > n) return 0;
  ld r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Multi-indices of degree n in the documented (graded) coefficient order: s = a1+a2+a3
// ascending, then a3, then a2; the degree-n list is a prefix of the degree-(n+1) list
// when compared by (a1, a2, a3).
std::vector<std::array<int, 4>> mi3_list(int n) {
  std::vector<std::array<int, 4>> out;
  for (int s = 0; s <= n; ++s)
    for (int a3 = 0; a3 <= s; ++a3)
      for (int a2 = 0; a2 <= s - a3; ++a2) out.push_back({n - s, s - a2 - a3, a2, a3});
  return out;
}

// ----------------------------------------------------------------- positivity
// Sign of a degree-m Bernstein polynomial on its tetrahedron. The Bernstein basis is a
// nonnegative partition of unity (Section 2), so the polynomial lies between its smallest
// and largest coefficient on the element, and the coefficient at a vertex (alpha = m e_i)
// is the value there. When neither decides, the tetrahedron is bisected at the midpoint of
// its longest edge (measured in barycentric coordinates); the coefficients of the two
// halves follow from univariate de Casteljau subdivision at t = 1/2 along that edge, and
// both halves are tested again. Returns +1 (positive everywhere), -1 (a value <= 0 was
// found at a vertex of a piece) or 0 (undecided after `budget` pieces).
int bernstein_sign(const double* coef, int m, int budget) {
  auto mi = mi3_list(m);
  const int np = (int)mi.size();
  if (m == 0) return coef[0] > 0 ? 1 : -1;
  // position of a multi-index given (a1, a2, a3) through a dense lookup
  std::vector<int> pos((size_t)(m + 1) * (m + 1) * (m + 1), -1);
  for (int i = 0; i < np; ++i) pos[((size_t)mi[i][1] * (m + 1) + mi[i][2]) * (m + 1) + mi[i][3]] = i;
  auto at = [&](int a1, int a2, int a3) { return pos[((size_t)a1 * (m + 1) + a2) * (m + 1) + a3]; };
  int vtx[4];
  vtx[0] = at(0, 0, 0), vtx[1] = at(m, 0, 0), vtx[2] = at(0, m, 0), vtx[3] = at(0, 0, m);
  struct Piece {
    std::vector<double> c;
    double v[4][4];  // barycentric coordinates (original element) of the piece's vertices
  };
  std::vector<Piece> stack;
  Piece root;
  root.c.assign(coef, coef + np);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) root.v[i][j] = i == j ? 1.0 : 0.0;
  stack.push_back(std::move(root));
  int used = 0;
  std::vector<double> line((size_t)m + 1), left((size_t)m + 1), right((size_t)m + 1);
  while (!stack.empty()) {
    Piece p = std::move(stack.back());
    stack.pop_back();
    for (int i = 0; i < 4; ++i)
      if (!(p.c[vtx[i]] > 0)) return -1;
    double lo = p.c[0];
    for (int i = 1; i < np; ++i) lo = std::min(lo, p.c[i]);
    if (lo > 0) continue;
    if (++used > budget) return 0;
    // longest edge of the piece
    int ei = 0, ej = 1;
    double best = -1;
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j) {
        double d = 0;
        for (int t = 0; t < 4; ++t) d += (p.v[i][t] - p.v[j][t]) * (p.v[i][t] - p.v[j][t]);
        if (d > best) best = d, ei = i, ej = j;
      }
    Piece A, B;
    A.c.assign(np, 0.0), B.c.assign(np, 0.0);
    std::memcpy(A.v, p.v, sizeof p.v), std::memcpy(B.v, p.v, sizeof p.v);
    for (int t = 0; t < 4; ++t) A.v[ej][t] = B.v[ei][t] = 0.5 * (p.v[ei][t] + p.v[ej][t]);
    // every line of coefficients with the other two indices fixed is a univariate
    // Bernstein polynomial in (lambda_ei, lambda_ej) of degree a_ei + a_ej
    for (int i = 0; i < np; ++i) {
      std::array<int, 4> a = mi[i];
      if (a[ej] != 0) continue;  // visit each line once, from its a_ej = 0 end
      const int len = a[ei];
      for (int k = 0; k <= len; ++k) {
        std::array<int, 4> b = a;
        b[ei] = len - k, b[ej] = k;
        line[k] = p.c[at(b[1], b[2], b[3])];
      }
      // de Casteljau at 1/2: left piece (ej moved to the midpoint) takes the first entry of
      // each level, right piece (ei moved) the last
      for (int r = 0; r <= len; ++r) {
        left[r] = line[0];
        right[len - r] = line[len - r];
        for (int k = 0; k < len - r; ++k) line[k] = 0.5 * (line[k] + line[k + 1]);
      }
      for (int k = 0; k <= len; ++k) {
        std::array<int, 4> b = a;
        b[ei] = len - k, b[ej] = k;
        const int q = at(b[1], b[2], b[3]);
        A.c[q] = left[k];
        B.c[q] = right[k];
      }
    }
    stack.push_back(std::move(A));
    stack.push_back(std::move(B));
  }
  return 1;
}

// ------------------------------------------------------------- projection coefficients
// Distinct eigenvalue k of the degree-n Bernstein mass matrix of the volume-4/3
// reference tetrahedron: (4/3) 3! (n!)^2 / ((n-k)! (n+k+3)!).
ld mass_eig(int n, int k) { return 8.0L * factl(n) * factl(n) / (factl(n - k) * factl(n + k + 3)); }

// c_j of the telescoped projection (paper Theorem 5.3). In the orthogonal modal basis
// E^N_{N-j}(E^N_{N-j})^T is diagonal with entries lambda^{N-j}_k / lambda^N_k on modes of
// degree k <= N-j (paper Corollary A.3) and the reduction (E^{N+M}_N)^T scales mode k by
// lambda^N_k / lambda^{N+M}_k (Lemma A.2), so requiring the identity on P^N gives the
// triangular system sum_{j=0}^{N-k} c_j lambda^{N-j}_k = lambda^{N+M}_k, k = N..0.
// With M < 0 the right-hand side is 1 (inverse mass matrix, Theorem 5.5).
void projection_cj(int N, int M, ld* c) {
  for (int k = N; k >= 0; --k) {
    int jn = N - k;
    ld rhs = (M < 0) ? 1.0L : mass_eig(N + M, k);
    ld s = 0;
    for (int j = 0; j < jn; ++j) s += c[j] * mass_eig(N - j, k);
    c[jn] = (rhs - s) / mass_eig(N - jn, k);
  }
}

// ----------------------------------------------------------------- Gauss-Jacobi rule
// Nodes: eigenvalues of the symmetric Jacobi matrix of the weight (1-x)^a (1+x)^b, found
// by bisection on Sturm sequence counts; weights: Christoffel numbers 1/sum_k p_k(x)^2
// with orthonormal p_k from the same three-term recurrence.
void gauss_jacobi(int n, ld a, ld b, std::vector<ld>& x, std::vector<ld>& w) {
  std::vector<ld> d(n), e2(n, 0);  // diagonal, squared off-diagonal (e2[i] couples i-1, i)
  for (int i = 0; i < n; ++i) {
    ld s = 2 * i + a + b;
    d[i] = (i == 0) ? (b - a) / (a + b + 2) : (b * b - a * a) / (s * (s + 2));
    if (i >= 1) e2[i] = 4.0L * i * (i + a) * (i + b) * (i + a + b) / (s * s * (s + 1) * (s - 1));
  }
  auto count_below = [&](ld lam) {  // number of eigenvalues < lam
    int cnt = 0;
    ld q = d[0] - lam;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
      if (q == 0) q = 1e-300L;
      q = d[i] - lam - e2[i] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  x.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    ld lo = -1, hi = 1;
    for (int it = 0; it < 200; ++it) {
      ld mid = 0.5L * (lo + hi);
      if (count_below(mid) > i) hi = mid; else lo = mid;
    }
    x[i] = 0.5L * (lo + hi);
  }
  ld mu0 = std::pow(2.0L, a + b + 1) * std::tgamma(a + 1) * std::tgamma(b + 1) / std::tgamma(a + b + 2);
  w.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    ld pm1 = 0, p = 1.0L / std::sqrt(mu0), sum = p * p;
    for (int k = 0; k + 1 < n; ++k) {
      ld pn = ((x[i] - d[k]) * p - (k > 0 ? std::sqrt(e2[k]) * pm1 : 0)) / std::sqrt(e2[k + 1]);
      pm1 = p;
      p = pn;
      sum += p * p;
    }
    w[i] = 1.0L / sum;
  }
}

// Collapsed rule on the reference tetrahedron, n points per direction; barycentric
// coordinates lam[q][4] and weights (sum = 4/3).
void tet_rule(int n, std::vector<std::array<ld, 4>>& lam, std::vector<ld>& w) {
  std::vector<ld> xa, wa, xb, wb, xc, wc;
  gauss_jacobi(n, 0, 0, xa, wa);
  gauss_jacobi(n, 1, 0, xb, wb);
  gauss_jacobi(n, 2, 0, xc, wc);
  lam.clear();
  w.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        ld A = xa[i], B = xb[j], C = xc[k];
        ld r = (1 + A) * (1 - B) * (1 - C) / 4 - 1;
        ld s = (1 + B) * (1 - C) / 2 - 1;
        ld t = C;
        lam.push_back({-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2});
        w.push_back(wa[i] * wb[j] * wc[k] / 8);
      }
}

ld bernstein(int n, const std::array<int, 4>& al, const std::array<ld, 4>& lam) {
  ld v = factl(n);
  for (int j = 0; j < 4; ++j) v = v / factl(al[j]) * std::pow(lam[j], (ld)al[j]);
  return v;
}

// Dense closed-form Bernstein mass matrix of degree n on the volume-4/3 tetrahedron:
// B_a B_b = C(a+b, a)/C(2n, n) B^{2n}_{a+b} and each degree-m Bernstein polynomial
// integrates to (4/3)/C(m+3, 3).
std::vector<ld> bernstein_mass(int n) {
  auto A = mi3_list(n);
  int np = (int)A.size();
  std::vector<ld> Mm((size_t)np * np);
  ld base = (4.0L / 3.0L) / (binoml(2 * n, n) * binoml(2 * n + 3, 3));
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      ld c = 1;
      for (int q = 0; q < 4; ++q) c *= binoml(A[i][q] + A[j][q], A[i][q]);
      Mm[(size_t)i * np + j] = c * base;
    }
  return Mm;
}

// Projection onto degree d from samples at the collapsed rule with d+3 points per
// direction: P = M_d^{-1} B^T W ([dimp(d)][nq], long-double Cholesky), plus B itself.
struct Projector {
  int degree = -1;
  int nq = 0;
  std::vector<double> P;     // [dimp][nq]
  std::vector<double> B;     // [nq][dimp] Bernstein values at the points
  std::vector<double> w;     // [nq] rule weights (sum 4/3)
  std::vector<std::array<ld, 4>> lam;
};

// Projection onto degree d with the collapsed rule of n points per direction.
void build_projector_rule(int d, int n, Projector& pr) {
  std::vector<ld> w;
  tet_rule(n, pr.lam, w);
  int nq = (int)w.size();
  auto A = mi3_list(d);
  int np = (int)A.size();
  std::vector<ld> Bq((size_t)nq * np);
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < np; ++i) Bq[(size_t)q * np + i] = bernstein(d, A[i], pr.lam[q]);
  std::vector<ld> L = bernstein_mass(d);
  // Cholesky L L^T = M
  for (int j = 0; j < np; ++j) {
    ld s = L[(size_t)j * np + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * np + k] * L[(size_t)j * np + k];
    ld djj = std::sqrt(s);
    L[(size_t)j * np + j] = djj;
    for (int i = j + 1; i < np; ++i) {
      ld t = L[(size_t)i * np + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * np + k] * L[(size_t)j * np + k];
      L[(size_t)i * np + j] = t / djj;
    }
  }
  pr.P.assign((size_t)np * nq, 0);
  std::vector<ld> col(np);
  for (int q = 0; q < nq; ++q) {
    for (int i = 0; i < np; ++i) col[i] = Bq[(size_t)q * np + i] * w[q];
    for (int i = 0; i < np; ++i) {  // forward
      ld t = col[i];
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * np + k] * col[k];
      col[i] = t / L[(size_t)i * np + i];
    }
    for (int i = np - 1; i >= 0; --i) {  // backward
      ld t = col[i];
      for (int k = i + 1; k < np; ++k) t -= L[(size_t)k * np + i] * col[k];
      col[i] = t / L[(size_t)i * np + i];
    }
    for (int i = 0; i < np; ++i) pr.P[(size_t)i * nq + q] = (double)col[i];
  }
  pr.B.assign((size_t)nq * np, 0);
  for (size_t i = 0; i < Bq.size(); ++i) pr.B[i] = (double)Bq[i];
  pr.w.assign(w.begin(), w.end());
  pr.degree = d;
  pr.nq = nq;
}

void build_projector(int d, Projector& pr) { build_projector_rule(d, d + 3, pr); }

// ------------------------------------------------------------------------ tables
// The stage kernel derives all its index maps from the graded coefficient order; the
// host only supplies the projection coefficients c_j.
struct HostTables {
  double cj[kMaxN + 1] = {0};
};

void build_tables(int N, int M, HostTables& T) {
  ld c[kMaxN + 1];
  projection_cj(N, M, c);
  for (int j = 0; j <= N; ++j) T.cj[j] = (double)c[j];
}

}  // namespace

int bbw::set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vfail(code, fmt, ap);
  va_end(ap);
  return code;
}

// ------------------------------------------------------------------------ context
struct bbwadg_ctx {
  int N = 0, M = 0, dtype = 0, mode = 0, bc = 0;
  double tau_p = 1, tau_u = 1;
  int64_t K = 0, Nv = 0;
  int Np = 0, Nfp = 0, Mp = 0;
  std::vector<double> xyz;
  std::vector<int32_t> etov;     // sorted per element
  std::vector<double> J;         // [K]
  std::vector<double> G;         // [K][9]
  std::vector<double> nrm;       // [K][4][3]
  std::vector<double> fscale;    // [K][4]
  std::vector<int32_t> conn;     // [K][4]
  std::vector<double> c2;        // [K][Mp]
  bool c2_set = false, c2_dirty = false;
  int c2_policy = BBWADG_C2_REQUIRE_POSITIVE;
  int64_t c2_nonpositive = 0, c2_undecided = 0;  // of the stored c^2_M
  HostTables tables;
  Projector proj[kMaxN + 1];
  // device
  int device = -1;
  size_t rsz = 8;
  void* d_geo = nullptr;
  void* d_conn = nullptr;
  void* d_c2 = nullptr;   // [K][Mp] c^2_M coefficients (dtype)
  void* d_c2k = nullptr;  // [K][Mp] c^2_M coefficients / beta! (dtype): the stage kernel's copy
  void* d_q2 = nullptr;
  void* d_J = nullptr;
  void* d_mass = nullptr;
  void* d_partial = nullptr;
  int nred_blocks = 0;
  // quadrature reductions: tables at the degree-N projection rule
  void* d_rbasis = nullptr;     // [Np][nq] B^N
  void* d_rbasis_c2 = nullptr;  // [Mp][nq] B^M
  void* d_rw = nullptr;         // [nq]
  int nq_red = 0;
  // dense quadrature WADG (comparison baseline)
  Projector dense;              // degree N at the dense rule: B = V_q, P = P_q
  int dense_n = 0, dense_nqp = 0;
  void* d_dva = nullptr;        // V_q in MFMA operand order (FP64; also the adjoint's)
  void* d_dpa = nullptr;        // P_q in MFMA operand order (FP64)
  void* d_dva32 = nullptr;      // the same tables in FP32 (FP32 contexts)
  void* d_dpa32 = nullptr;
  void* d_c2q = nullptr;        // [K][dense_nqp] c^2 at the dense points
  void* d_ones = nullptr;       // [K] ones of the context dtype: c^2 = 1 for the plain DG right-hand side
  bool c2q_set = false;
  // pressure source f(x, t) = amp sin(omega t + phase) g(x)
  void* d_src = nullptr;        // [K][Np] coefficients of g (dtype)
  double src_amp = 0, src_omega = 0, src_phase = 0;
  // receivers (pressure samples) and the misfit gradient
  int32_t nrec = 0;
  std::vector<int32_t> rec_elem;      // [nrec] containing element
  std::vector<double> rec_basis;      // [nrec][Np] B^N_alpha at the receiver
  std::vector<double> rec_kvec;       // [nrec][Np] (J_k M)^{-1} of that row
  void* d_rec_elem = nullptr;
  void* d_rec_basis = nullptr;
  void* d_rec_kvec = nullptr;
  void* d_adj_bwa = nullptr;    // rule weight times B^M at the dense points, MFMA operand order
  void* d_adj_ones = nullptr;   // [K] ones (dtype): c^2 = 1 for the plain DG operator
  // elastic media (isotropic): Bernstein coefficients of degree M, dtype
  void* d_el_rho = nullptr;     // [K][Mp] 1/rho
  void* d_el_lam = nullptr;     // [K][Mp] lambda
  void* d_el_mu = nullptr;      // [K][Mp] mu
  void* d_el_fpos = nullptr;    // [4][Nfp] int32
  void* d_el_tmp = nullptr;     // [9][K][Np] pre-update right-hand side (dtype)
  void* d_el_rhs = nullptr;     // [9][K][Np] weighted right-hand side of a time step, N >= 8 (dtype)
};

namespace {

// Split [a, b) over hardware threads (setup-time host loops only).
template <typename F>
void parallel_for(int64_t a, int64_t b, F&& fn) {
  int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
  if (b - a < 256) nt = 1;
  if (nt == 1) { fn(a, b); return; }
  std::vector<std::thread> th;
  int64_t chunk = (b - a + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t lo = a + t * chunk, hi = std::min(b, lo + chunk);
    if (lo < hi) th.emplace_back([&fn, lo, hi] { fn(lo, hi); });
  }
  for (auto& x : th) x.join();
}

const Projector& get_projector(const bbwadg_ctx* ctx, int d) {
  auto* c = const_cast<bbwadg_ctx*>(ctx);
  if (c->proj[d].degree != d) build_projector(d, c->proj[d]);
  return c->proj[d];
}

void free_device(bbwadg_ctx* c) {
  void** ptrs[] = {&c->d_geo,     &c->d_conn,    &c->d_c2,         &c->d_c2k, &c->d_q2,
                   &c->d_J,       &c->d_mass,    &c->d_partial,    &c->d_rbasis, &c->d_rbasis_c2,
                   &c->d_rw,      &c->d_dva,     &c->d_dpa,        &c->d_c2q, &c->d_ones, &c->d_dva32, &c->d_dpa32,
                   &c->d_src,     &c->d_rec_elem, &c->d_rec_basis, &c->d_rec_kvec, &c->d_adj_bwa,
                   &c->d_adj_ones, &c->d_el_rho, &c->d_el_lam, &c->d_el_mu, &c->d_el_fpos, &c->d_el_tmp, &c->d_el_rhs};
  for (void** p : ptrs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
}

template <typename real>
std::vector<real> convert(const std::vector<double>& v) {
  return std::vector<real>(v.begin(), v.end());
}

int upload(void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  return e == hipSuccess ? 0 : fail(BBWADG_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
}

int dmalloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 8);
  return e == hipSuccess ? 0 : fail(BBWADG_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
}

// Classification of n sets of degree-m Bernstein coefficients [n][dimp(m)]: counts of sets
// that are not positive everywhere on their element (a value <= 0 found) and of sets whose
// sign the subdivision budget could not decide. EC2 if a coefficient is not finite.
struct PositivityCount {
  int64_t nonpositive = 0, undecided = 0, first = -1;
};
constexpr int kSignBudget = 4096;  // pieces per element before a set counts as undecided

int classify_positive(const double* coef, int m, int64_t n, PositivityCount& out, const char* what) {
  const int mp = dimp(m);
  for (int64_t i = 0; i < n * mp; ++i)
    if (!std::isfinite(coef[i]))
      return fail(BBWADG_EC2, "%s coefficient of element %lld not finite", what, (long long)(i / mp));
  std::atomic<int64_t> nonpos{0}, undec{0}, first{std::numeric_limits<int64_t>::max()};
  parallel_for(0, n, [&](int64_t a, int64_t b) {
    int64_t np_ = 0, ud = 0, f = std::numeric_limits<int64_t>::max();
    for (int64_t k = a; k < b; ++k) {
      const int sg = bernstein_sign(coef + k * mp, m, kSignBudget);
      if (sg < 0) ++np_;
      if (sg == 0) ++ud;
      if (sg <= 0 && k < f) f = k;
    }
    nonpos += np_;
    undec += ud;
    int64_t cur = first.load();
    while (f < cur && !first.compare_exchange_weak(cur, f)) {
    }
  });
  out.nonpositive = nonpos.load();
  out.undecided = undec.load();
  out.first = out.nonpositive + out.undecided > 0 ? first.load() : -1;
  return 0;
}

// c^2_M must be finite, and positive everywhere on every element (the weight of the
// weight-adjusted mass matrix, Section 3) unless the context's policy accepts otherwise.
int check_c2(bbwadg_ctx* ctx, const double* coef) {
  PositivityCount pc;
  int rc = classify_positive(coef, ctx->M, ctx->K, pc, "c^2");
  if (rc) return rc;
  if (ctx->c2_policy == BBWADG_C2_REQUIRE_POSITIVE && pc.nonpositive + pc.undecided > 0)
    return fail(BBWADG_EC2,
                "c^2_M is not positive everywhere on %lld elements (%lld with a value <= 0, %lld undecided; "
                "first element %lld)",
                (long long)(pc.nonpositive + pc.undecided), (long long)pc.nonpositive, (long long)pc.undecided,
                (long long)pc.first);
  ctx->c2_nonpositive = pc.nonpositive;
  ctx->c2_undecided = pc.undecided;
  return 0;
}

// Upload c^2_M (as stored) and the stage kernel's copy scaled by 1/beta!: the product of
// eq. (mcoeff) is evaluated in that scaled form.
int sync_c2(bbwadg_ctx* ctx, hipStream_t s) {
  if (!ctx->c2_set) return fail(BBWADG_EC2, "c^2 not set (call bbwadg_project_c2 or bbwadg_set_c2)");
  if (!ctx->c2_dirty) return 0;
  const int mp = ctx->Mp;
  auto B = mi3_list(ctx->M);
  std::vector<double> inv(mp);
  for (int b = 0; b < mp; ++b)
    inv[b] = (double)(1.0L / (factl(B[b][0]) * factl(B[b][1]) * factl(B[b][2]) * factl(B[b][3])));
  std::vector<double> scaled(ctx->c2.size());
  for (size_t i = 0; i < scaled.size(); ++i) scaled[i] = ctx->c2[i] * inv[i % mp];
  hipError_t e;
  if (ctx->dtype == BBWADG_F64) {
    e = hipMemcpyAsync(ctx->d_c2, ctx->c2.data(), ctx->c2.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->d_c2k, scaled.data(), scaled.size() * 8, hipMemcpyHostToDevice, s);
  } else {
    std::vector<float> f = convert<float>(ctx->c2), fk = convert<float>(scaled);
    e = hipMemcpyAsync(ctx->d_c2, f.data(), f.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->d_c2k, fk.data(), fk.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // f, fk are local buffers
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // scaled is a local buffer
  if (e != hipSuccess) return fail(BBWADG_EHIP, "c^2 upload: %s", hipGetErrorString(e));
  ctx->c2_dirty = false;
  return 0;
}

// The c_j of the telescoped projection for a kernel's argument block, in the kernel's
// precision and in FP64.
template <typename Args>
void set_cj(const bbwadg_ctx* c, Args& a) {
  using real = std::remove_reference_t<decltype(a.cj[0])>;
  for (int j = 0; j <= kMaxN; ++j) {
    a.cj[j] = (real)c->tables.cj[j];
    a.cjd[j] = (double)c->tables.cj[j];
  }
}

template <typename real>
StageArgs<real> make_args(const bbwadg_ctx* c) {
  StageArgs<real> a{};
  a.geo = (const real*)c->d_geo;
  a.conn = (const int32_t*)c->d_conn;
  a.c2 = (const real*)c->d_c2k;
  a.K = c->K;
  a.tau_p = (real)c->tau_p;
  a.tau_u = (real)c->tau_u;
  a.bc = c->bc;
  set_cj(c, a);
  a.src = (const real*)c->d_src;
  a.src_amp = real(0);
  a.rp_out = nullptr;
  return a;
}

// s(t) of the pressure source at time t (0 without a source).
double source_factor(const bbwadg_ctx* c, double t) {
  return c->d_src ? c->src_amp * std::sin(c->src_omega * t + c->src_phase) : 0.0;
}

const double kRkA[5] = {0.0,
                        -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double kRkC[5] = {0.0,
                        1432997174477.0 / 9575080441755.0,
                        2526269341429.0 / 6820363183787.0,
                        2006345519317.0 / 3224310063776.0,
                        2802321613138.0 / 2924317926251.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0,
                        5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0,
                        3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

int launch(bbwadg_ctx* c, bool update, const void* qin, void* qout, void* res, double ra, double rb,
           double dt, double t, hipStream_t s, void* rp_out = nullptr) {
  int e;
  const double sf = source_factor(c, t);
  if (c->dtype == BBWADG_F64) {
    StageArgs<double> a = make_args<double>(c);
    a.rp_out = (double*)rp_out;
    a.src_amp = sf;
    a.qin = (const double*)qin;
    a.qout = (double*)qout;
    a.res = (double*)res;
    a.rk_a = ra;
    a.rk_b = rb;
    a.dt = dt;
    e = launch_stage_f64(c->N, c->M, update, a, s);
  } else {
    StageArgs<float> a = make_args<float>(c);
    a.rp_out = (float*)rp_out;
    a.src_amp = (float)sf;
    a.qin = (const float*)qin;
    a.qout = (float*)qout;
    a.res = (float*)res;
    a.rk_a = (float)ra;
    a.rk_b = (float)rb;
    a.dt = (float)dt;
    e = launch_stage_f32(c->N, c->M, update, a, s);
  }
  if (e != 0) return fail(BBWADG_EHIP, "stage launch: %s", hipGetErrorString((hipError_t)e));
  return 0;
}

// One quadrature reduction over elements [k0, k1) (mode 0: error, 1: energy); sums the
// per-block partials on the host in block order.
int quad_reduce(bbwadg_ctx* c, int mode, const void* q, int64_t k0, int64_t k1, const double* exact, double out[4],
                hipStream_t s) {
  if (k0 < 0 || k1 > c->K || k0 > k1) return fail(BBWADG_EINVAL, "bad element range");
  for (int f = 0; f < 4; ++f) out[f] = 0.0;
  if (k0 == k1) return 0;
  QuadReduceArgs a{};
  a.q = q;
  a.c2 = c->d_c2;
  a.J = (const double*)c->d_J;
  a.basis = (const double*)c->d_rbasis;
  a.basis_c2 = (const double*)c->d_rbasis_c2;
  a.w = (const double*)c->d_rw;
  a.exact = exact;
  a.partial = (double*)c->d_partial;
  a.K = c->K;
  a.k0 = k0;
  a.k1 = k1;
  a.Np = c->Np;
  a.Mp = c->Mp;
  a.nq = c->nq_red;
  const int nb = quad_reduce_blocks(k1 - k0, c->nred_blocks);
  int e = launch_quad_reduce(c->dtype, mode, a, nb, s);
  if (e) return fail(BBWADG_EHIP, "reduction launch: %s", hipGetErrorString((hipError_t)e));
  std::vector<double> part((size_t)nb * 4);
  hipError_t he = hipMemcpyAsync(part.data(), c->d_partial, part.size() * 8, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return fail(BBWADG_EHIP, "reduction copy: %s", hipGetErrorString(he));
  for (int f = 0; f < 4; ++f) {
    double acc = 0;
    for (int b = 0; b < nb; ++b) acc += part[(size_t)b * 4 + f];
    out[f] = acc;
  }
  return 0;
}

// Points per direction of the dense WADG rule: exact for degree 2N+M, so that with c^2_M
// at the points the dense update is the exact projection (the fast method's result).
int dense_rule_n(const bbwadg_ctx* c) { return (2 * c->N + c->M + 2) / 2; }

const Projector& get_dense(bbwadg_ctx* c) {
  const int n = dense_rule_n(c);
  if (c->dense_n != n) {
    build_projector_rule(c->N, n, c->dense);
    c->dense_n = n;
    c->dense_nqp = (c->dense.nq + 15) / 16 * 16;
  }
  return c->dense;
}

// Upload V_q and P_q in MFMA operand order (zero padded), once.
int dense_tables(bbwadg_ctx* c) {
  if (c->d_dva) return 0;
  const Projector& pr = get_dense(c);
  const int np = c->Np, nq = pr.nq, npp = (np + 15) / 16 * 16, nqp = c->dense_nqp;
  const int nqc = nqp / 16, nk = npp / 4, nt = npp / 16;
  std::vector<double> va((size_t)nqc * nk * 64, 0.0), pa((size_t)nqc * nt * 4 * 64, 0.0);
  for (int qc = 0; qc < nqc; ++qc)
    for (int l = 0; l < 64; ++l) {
      for (int ks = 0; ks < nk; ++ks) {
        const int q = 16 * qc + l % 16, i = 4 * ks + l / 16;
        va[((size_t)qc * nk + ks) * 64 + l] = (q < nq && i < np) ? pr.B[(size_t)q * np + i] : 0.0;
      }
      for (int t = 0; t < nt; ++t)
        for (int ks = 0; ks < 4; ++ks) {
          const int i = 16 * t + l % 16, q = 16 * qc + 4 * ks + l / 16;
          pa[(((size_t)qc * nt + t) * 4 + ks) * 64 + l] = (q < nq && i < np) ? pr.P[(size_t)i * nq + q] : 0.0;
        }
    }
  std::vector<double> ones((size_t)c->K, 1.0);
  const bool f32 = c->dtype == BBWADG_F32;
  int rc = dmalloc(&c->d_dva, va.size() * 8);
  if (!rc) rc = dmalloc(&c->d_dpa, pa.size() * 8);
  if (!rc) rc = dmalloc(&c->d_ones, ones.size() * c->rsz);
  if (!rc) rc = upload(c->d_dva, va.data(), va.size() * 8);
  if (!rc) rc = upload(c->d_dpa, pa.data(), pa.size() * 8);
  if (!rc && !f32) rc = upload(c->d_ones, ones.data(), ones.size() * 8);
  if (!rc && f32) {
    std::vector<float> va32 = convert<float>(va), pa32 = convert<float>(pa), ones32 = convert<float>(ones);
    rc = dmalloc(&c->d_dva32, va32.size() * 4);
    if (!rc) rc = dmalloc(&c->d_dpa32, pa32.size() * 4);
    if (!rc) rc = upload(c->d_dva32, va32.data(), va32.size() * 4);
    if (!rc) rc = upload(c->d_dpa32, pa32.data(), pa32.size() * 4);
    if (!rc) rc = upload(c->d_ones, ones32.data(), ones32.size() * 4);
  }
  if (rc) {
    void** ptrs[] = {&c->d_dva, &c->d_dpa, &c->d_ones, &c->d_dva32, &c->d_dpa32};
    for (void** p : ptrs) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
  }
  return rc;
}

int require_device(const bbwadg_ctx* c) {
  if (!c) return fail(BBWADG_EINVAL, "NULL context");
  if (c->mode != BBWADG_DEVICE) return fail(BBWADG_EINVAL, "host-only context");
  return 0;
}

}  // namespace

// ------------------------------------------------------------------------- C ABI
extern "C" {

const char* bbwadg_last_error(void) { return g_err.c_str(); }
const char* bbwadg_version(void) { return "bbwadg-mi355x 0.1"; }

int bbwadg_projection_coefficients(int32_t N, int32_t M, double* cj_out) {
  if (N < 1 || N > kMaxN || M < -1 || M > 9 || !cj_out) return fail(BBWADG_EINVAL, "bad N/M");
  ld c[kMaxN + 1];
  projection_cj(N, M, c);
  for (int j = 0; j <= N; ++j) cj_out[j] = (double)c[j];
  return 0;
}

int bbwadg_create(const bbwadg_mesh* mesh, const bbwadg_opts* opts, bbwadg_ctx** out) {
  g_err.clear();
  if (!mesh || !opts || !out) return fail(BBWADG_EINVAL, "NULL argument");
  *out = nullptr;
  const int N = opts->N, M = opts->M;
  if (N < 1 || N > kMaxN) return fail(BBWADG_EINVAL, "N=%d outside [1,%d]", N, kMaxN);
  if (M < 0 || M > std::min(N, kMaxM)) return fail(BBWADG_EINVAL, "M=%d outside [0,min(N,%d)]", M, kMaxM);
  if (opts->dtype != BBWADG_F64 && opts->dtype != BBWADG_F32) return fail(BBWADG_EINVAL, "bad dtype");
  if (opts->mode != BBWADG_DEVICE && opts->mode != BBWADG_HOST_ONLY) return fail(BBWADG_EINVAL, "bad mode");
  if (!(opts->tau_p >= 0) || !(opts->tau_u >= 0) || !std::isfinite(opts->tau_p) || !std::isfinite(opts->tau_u))
    return fail(BBWADG_EINVAL, "tau must be finite and >= 0");
  if (mesh->bc != BBWADG_BC_P0 && mesh->bc != BBWADG_BC_RIGID) return fail(BBWADG_EINVAL, "bad bc");
  if (mesh->num_elements < 1 || mesh->num_vertices < 4 || !mesh->xyz || !mesh->etov)
    return fail(BBWADG_EINVAL, "empty mesh or NULL arrays");
  if (mesh->num_elements > (int64_t)1 << 28) return fail(BBWADG_EINVAL, "too many elements");
  const int64_t K = mesh->num_elements, Nv = mesh->num_vertices;

  bbwadg_ctx* c = new (std::nothrow) bbwadg_ctx();
  if (!c) return fail(BBWADG_ENOMEM, "context");
  c->N = N; c->M = M; c->dtype = opts->dtype; c->mode = opts->mode; c->bc = mesh->bc;
  c->tau_p = opts->tau_p; c->tau_u = opts->tau_u;
  c->K = K; c->Nv = Nv;
  c->Np = dimp(N); c->Nfp = dim2(N); c->Mp = dimp(M);
  c->rsz = (c->dtype == BBWADG_F64) ? 8 : 4;
  c->xyz.assign(mesh->xyz, mesh->xyz + 3 * Nv);
  c->etov.resize(4 * K);
  for (int64_t k = 0; k < K; ++k) {
    int32_t v[4];
    for (int j = 0; j < 4; ++j) {
      v[j] = mesh->etov[4 * k + j];
      if (v[j] < 0 || v[j] >= Nv) { delete c; return fail(BBWADG_EINVAL, "vertex id out of range in element %lld", (long long)k); }
    }
    std::sort(v, v + 4);
    if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) { delete c; return fail(BBWADG_EMESH, "repeated vertex in element %lld", (long long)k); }
    for (int j = 0; j < 4; ++j) c->etov[4 * k + j] = v[j];
  }
  // geometry
  c->J.resize(K); c->G.resize(9 * K); c->nrm.resize(12 * K); c->fscale.resize(4 * K);
  for (int64_t k = 0; k < K; ++k) {
    double V[4][3];
    for (int j = 0; j < 4; ++j)
      for (int d = 0; d < 3; ++d) V[j][d] = c->xyz[3 * (size_t)c->etov[4 * k + j] + d];
    double A[3][3];  // A[i][j] = d x_i / d r_j
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[i][j] = 0.5 * (V[j + 1][i] - V[0][i]);
    double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                 A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    double h = 0;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        double d2 = 0;
        for (int d = 0; d < 3; ++d) d2 += (V[a][d] - V[b][d]) * (V[a][d] - V[b][d]);
        h = std::max(h, std::sqrt(d2));
      }
    if (!(std::fabs(det) > 1e-14 * h * h * h)) { delete c; return fail(BBWADG_EMESH, "degenerate element %lld", (long long)k); }
    double inv[3][3];  // inverse of A: inv[j][i] = d r_j / d x_i
    inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    double J = std::fabs(det);
    c->J[k] = J;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) c->G[9 * k + 3 * i + j] = inv[j][i];
    for (int f = 0; f < 4; ++f) {
      int u[3], m = 0;
      for (int v = 0; v < 4; ++v)
        if (v != f) u[m++] = v;
      double e1[3], e2[3], cr[3];
      for (int d = 0; d < 3; ++d) { e1[d] = V[u[1]][d] - V[u[0]][d]; e2[d] = V[u[2]][d] - V[u[0]][d]; }
      cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
      cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
      cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
      double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      double dotv = 0;
      for (int d = 0; d < 3; ++d) dotv += cr[d] * (V[u[0]][d] - V[f][d]);
      double sg = dotv > 0 ? 1.0 : -1.0;
      for (int d = 0; d < 3; ++d) c->nrm[12 * k + 3 * f + d] = sg * cr[d] / len;
      double area = 0.5 * len;
      c->fscale[4 * k + f] = (area / 2.0) / J;
    }
  }
  // connectivity: match faces by their sorted global vertex triple
  {
    struct Key { int32_t a, b, c; bool operator==(const Key& o) const { return a == o.a && b == o.b && c == o.c; } };
    struct H { size_t operator()(const Key& k) const { return ((size_t)k.a * 0x9E3779B97F4A7C15ull) ^ ((size_t)k.b * 0xC2B2AE3D27D4EB4Full) ^ ((size_t)k.c * 0x165667B19E3779F9ull); } };
    std::unordered_map<Key, int64_t, H> faces;
    faces.reserve((size_t)(2.5 * K) + 16);
    c->conn.assign(4 * K, -1);
    for (int64_t k = 0; k < K; ++k)
      for (int f = 0; f < 4; ++f) {
        int32_t u[3], m = 0;
        for (int v = 0; v < 4; ++v)
          if (v != f) u[m++] = c->etov[4 * k + v];
        Key key{u[0], u[1], u[2]};  // already ascending
        auto it = faces.find(key);
        if (it == faces.end()) {
          faces.emplace(key, 4 * k + f);
        } else {
          int64_t other = it->second;
          if (other < 0) { delete c; return fail(BBWADG_EMESH, "face shared by more than two elements (element %lld)", (long long)k); }
          c->conn[4 * k + f] = (int32_t)other;
          c->conn[other] = (int32_t)(4 * k + f);
          it->second = -1;
        }
      }
  }
  build_tables(N, M, c->tables);
  if (c->mode == BBWADG_HOST_ONLY) { *out = c; return 0; }

  // device buffers
  int rc = 0;
  hipError_t he = hipGetDevice(&c->device);
  if (he != hipSuccess) { delete c; return fail(BBWADG_EHIP, "hipGetDevice: %s", hipGetErrorString(he)); }
  std::vector<double> geo((size_t)K * kGeoStride);
  for (int64_t k = 0; k < K; ++k) {
    double* g = &geo[(size_t)k * kGeoStride];
    for (int i = 0; i < 9; ++i) g[i] = c->G[9 * k + i];
    for (int f = 0; f < 4; ++f) {
      g[9 + 4 * f] = c->fscale[4 * k + f];
      for (int d = 0; d < 3; ++d) g[9 + 4 * f + 1 + d] = c->nrm[12 * k + 3 * f + d];
    }
  }
  size_t rs = c->rsz;
  const size_t qbytes = (size_t)4 * K * c->Np * rs;
  c->nred_blocks = 1024;
  if ((rc = dmalloc(&c->d_geo, geo.size() * rs)) || (rc = dmalloc(&c->d_conn, c->conn.size() * 4)) ||
      (rc = dmalloc(&c->d_c2, (size_t)K * c->Mp * rs)) || (rc = dmalloc(&c->d_c2k, (size_t)K * c->Mp * rs)) ||
      (rc = dmalloc(&c->d_q2, qbytes)) ||
      (rc = dmalloc(&c->d_J, (size_t)K * 8)) || (rc = dmalloc(&c->d_mass, (size_t)c->Np * c->Np * 8)) ||
      (rc = dmalloc(&c->d_partial, (size_t)c->nred_blocks * 4 * 8))) {
    free_device(c);
    delete c;
    return rc;
  }
  // the fixed scratch array of the allocation-free entry points, resolved on this device
  if (int se = scratch_init()) {
    free_device(c);
    delete c;
    return fail(BBWADG_EHIP, "scratch address: %s", hipGetErrorString((hipError_t)se));
  }
  std::vector<ld> mass = bernstein_mass(N);
  std::vector<double> massd(mass.begin(), mass.end());
  if (rs == 8) {
    rc = upload(c->d_geo, geo.data(), geo.size() * 8);
  } else {
    std::vector<float> gf = convert<float>(geo);
    rc = upload(c->d_geo, gf.data(), gf.size() * 4);
  }
  if (!rc) rc = upload(c->d_conn, c->conn.data(), c->conn.size() * 4);
  if (!rc) rc = upload(c->d_J, c->J.data(), (size_t)K * 8);
  if (!rc) rc = upload(c->d_mass, massd.data(), massd.size() * 8);
  if (!rc) {
    // tables of the quadrature reductions: the degree-N projection rule, B^N and B^M there
    const Projector& pr = get_projector(c, N);
    const int nq = pr.nq, np = c->Np, mp = c->Mp;
    auto AM = mi3_list(M);
    std::vector<double> bt((size_t)np * nq), bm((size_t)mp * nq);
    for (int qq = 0; qq < nq; ++qq) {
      for (int i = 0; i < np; ++i) bt[(size_t)i * nq + qq] = pr.B[(size_t)qq * np + i];
      for (int i = 0; i < mp; ++i) bm[(size_t)i * nq + qq] = (double)bernstein(M, AM[i], pr.lam[qq]);
    }
    c->nq_red = nq;
    rc = dmalloc(&c->d_rbasis, bt.size() * 8);
    if (!rc) rc = dmalloc(&c->d_rbasis_c2, bm.size() * 8);
    if (!rc) rc = dmalloc(&c->d_rw, (size_t)nq * 8);
    if (!rc) rc = upload(c->d_rbasis, bt.data(), bt.size() * 8);
    if (!rc) rc = upload(c->d_rbasis_c2, bm.data(), bm.size() * 8);
    if (!rc) rc = upload(c->d_rw, pr.w.data(), (size_t)nq * 8);
  }
  if (rc) { free_device(c); delete c; return rc; }
  *out = c;
  return 0;
}

int bbwadg_destroy(bbwadg_ctx* ctx) {
  if (!ctx) return 0;
  if (ctx->mode == BBWADG_DEVICE) {
    (void)hipDeviceSynchronize();
    free_device(ctx);
  }
  delete ctx;
  return 0;
}

int bbwadg_sizes(const bbwadg_ctx* c, int32_t* Np, int32_t* Nfp, int32_t* Mp, int64_t* K) {
  if (!c) return fail(BBWADG_EINVAL, "NULL context");
  if (Np) *Np = c->Np;
  if (Nfp) *Nfp = c->Nfp;
  if (Mp) *Mp = c->Mp;
  if (K) *K = c->K;
  return 0;
}

int bbwadg_element_vertices(const bbwadg_ctx* c, int32_t* etov_out) {
  if (!c || !etov_out) return fail(BBWADG_EINVAL, "NULL argument");
  std::memcpy(etov_out, c->etov.data(), c->etov.size() * 4);
  return 0;
}

int bbwadg_geometry(const bbwadg_ctx* c, double* J, double* G, double* normal, double* Fscale, int32_t* nbr) {
  if (!c) return fail(BBWADG_EINVAL, "NULL context");
  if (J) std::memcpy(J, c->J.data(), c->J.size() * 8);
  if (G) std::memcpy(G, c->G.data(), c->G.size() * 8);
  if (normal) std::memcpy(normal, c->nrm.data(), c->nrm.size() * 8);
  if (Fscale) std::memcpy(Fscale, c->fscale.data(), c->fscale.size() * 8);
  if (nbr) std::memcpy(nbr, c->conn.data(), c->conn.size() * 4);
  return 0;
}

int bbwadg_projection_npoints(const bbwadg_ctx* c, int32_t degree, int64_t* nq) {
  if (!c || !nq) return fail(BBWADG_EINVAL, "NULL argument");
  if (degree < 0 || degree > kMaxN) return fail(BBWADG_EINVAL, "degree outside [0,%d]", kMaxN);
  *nq = (int64_t)(degree + 3) * (degree + 3) * (degree + 3);
  return 0;
}

int bbwadg_projection_points(const bbwadg_ctx* c, int32_t degree, int64_t k0, int64_t k1, double* xyz_out) {
  if (!c || !xyz_out) return fail(BBWADG_EINVAL, "NULL argument");
  if (degree < 0 || degree > kMaxN) return fail(BBWADG_EINVAL, "degree outside [0,%d]", kMaxN);
  if (k0 < 0 || k1 > c->K || k0 > k1) return fail(BBWADG_EINVAL, "bad element range");
  const Projector& pr = get_projector(c, degree);
  for (int64_t k = k0; k < k1; ++k) {
    const int32_t* v = &c->etov[4 * k];
    for (int q = 0; q < pr.nq; ++q)
      for (int d = 0; d < 3; ++d) {
        ld x = 0;
        for (int j = 0; j < 4; ++j) x += pr.lam[q][j] * (ld)c->xyz[3 * (size_t)v[j] + d];
        xyz_out[((size_t)(k - k0) * pr.nq + q) * 3 + d] = (double)x;
      }
  }
  return 0;
}

int bbwadg_project_samples(const bbwadg_ctx* c, int32_t degree, int64_t k0, int64_t k1, const double* samples,
                           double* coef_out) {
  if (!c || !samples || !coef_out) return fail(BBWADG_EINVAL, "NULL argument");
  if (degree < 0 || degree > kMaxN) return fail(BBWADG_EINVAL, "degree outside [0,%d]", kMaxN);
  if (k0 < 0 || k1 > c->K || k0 > k1) return fail(BBWADG_EINVAL, "bad element range");
  const Projector& pr = get_projector(c, degree);
  const int np = dimp(degree), nq = pr.nq;
  auto work = [&](int64_t a, int64_t b) {
    for (int64_t k = a; k < b; ++k) {
      const double* s = samples + (size_t)(k - k0) * nq;
      double* o = coef_out + (size_t)(k - k0) * np;
      for (int i = 0; i < np; ++i) {
        const double* P = &pr.P[(size_t)i * nq];
        double acc = 0;
        for (int q = 0; q < nq; ++q) acc += P[q] * s[q];
        o[i] = acc;
      }
    }
  };
  parallel_for(k0, k1, work);
  return 0;
}

int bbwadg_set_c2(bbwadg_ctx* c, const double* coef) {
  if (!c || !coef) return fail(BBWADG_EINVAL, "NULL argument");
  int rc = check_c2(c, coef);
  if (rc) return rc;
  c->c2.assign(coef, coef + (size_t)c->K * c->Mp);
  c->c2_set = true;
  c->c2_dirty = true;
  return 0;
}

int bbwadg_set_c2_policy(bbwadg_ctx* c, int32_t policy) {
  if (!c) return fail(BBWADG_EINVAL, "NULL context");
  if (policy != BBWADG_C2_REQUIRE_POSITIVE && policy != BBWADG_C2_ACCEPT_NONPOSITIVE)
    return fail(BBWADG_EINVAL, "unknown c^2 policy %d", (int)policy);
  c->c2_policy = policy;
  return 0;
}

int bbwadg_c2_positivity(const bbwadg_ctx* c, int64_t* n_nonpositive, int64_t* n_undecided) {
  if (!c) return fail(BBWADG_EINVAL, "NULL context");
  if (!c->c2_set) return fail(BBWADG_EC2, "c^2 not set");
  if (n_nonpositive) *n_nonpositive = c->c2_nonpositive;
  if (n_undecided) *n_undecided = c->c2_undecided;
  return 0;
}

int bbwadg_bernstein_positivity(int32_t degree, int64_t n, const double* coef, int64_t* n_nonpositive,
                                int64_t* n_undecided, int64_t* first) {
  if (degree < 0 || degree > kMaxDeg || n < 0 || (n > 0 && !coef)) return fail(BBWADG_EINVAL, "bad argument");
  PositivityCount pc;
  int rc = classify_positive(coef, degree, n, pc, "Bernstein");
  if (rc) return rc;
  if (n_nonpositive) *n_nonpositive = pc.nonpositive;
  if (n_undecided) *n_undecided = pc.undecided;
  if (first) *first = pc.first;
  return 0;
}

int bbwadg_get_c2(const bbwadg_ctx* c, double* coef) {
  if (!c || !coef) return fail(BBWADG_EINVAL, "NULL argument");
  if (!c->c2_set) return fail(BBWADG_EC2, "c^2 not set");
  std::memcpy(coef, c->c2.data(), c->c2.size() * 8);
  return 0;
}

int bbwadg_project_c2(bbwadg_ctx* c, double (*fn)(double, double, double, void*), void* user, void* c2_out,
                      void* stream) {
  if (!c || !fn) return fail(BBWADG_EINVAL, "NULL argument");
  if (c2_out && c->mode != BBWADG_DEVICE) return fail(BBWADG_EINVAL, "c2_out needs a device context");
  const Projector& pr = get_projector(c, c->M);
  const int64_t K = c->K;
  std::vector<double> coef((size_t)K * c->Mp);
  const int64_t chunk = 4096;
  std::vector<double> xyz, smp;
  for (int64_t k0 = 0; k0 < K; k0 += chunk) {
    int64_t k1 = std::min(K, k0 + chunk);
    xyz.resize((size_t)(k1 - k0) * pr.nq * 3);
    smp.resize((size_t)(k1 - k0) * pr.nq);
    int rc = bbwadg_projection_points(c, c->M, k0, k1, xyz.data());
    if (rc) return rc;
    for (size_t i = 0; i < smp.size(); ++i) smp[i] = fn(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], user);
    rc = bbwadg_project_samples(c, c->M, k0, k1, smp.data(), &coef[(size_t)k0 * c->Mp]);
    if (rc) return rc;
  }
  int rc = bbwadg_set_c2(c, coef.data());
  if (rc) return rc;
  if (c2_out) {
    hipStream_t s = (hipStream_t)stream;
    rc = sync_c2(c, s);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(c2_out, c->d_c2, (size_t)K * c->Mp * c->rsz, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(BBWADG_EHIP, "c2 copy: %s", hipGetErrorString(e));
  }
  return 0;
}

int bbwadg_rhs(bbwadg_ctx* c, const void* q, void* rhs, double t, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !rhs) return fail(BBWADG_EINVAL, "NULL state pointer");
  if (q == rhs) return fail(BBWADG_EINVAL, "q and rhs must not overlap");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = sync_c2(c, s))) return rc;
  return launch(c, false, q, rhs, nullptr, 0.0, 0.0, 0.0, t, s);
}

int bbwadg_step(bbwadg_ctx* c, void* q, void* res, double t0, double dt, int32_t nsteps, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !res) return fail(BBWADG_EINVAL, "NULL state pointer");
  if (q == res) return fail(BBWADG_EINVAL, "q and res must not overlap");
  if (nsteps < 0 || !std::isfinite(dt) || !std::isfinite(t0)) return fail(BBWADG_EINVAL, "bad nsteps, dt or t0");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = sync_c2(c, s))) return rc;
  void* cur = q;
  void* nxt = c->d_q2;
  for (int32_t n = 0; n < nsteps; ++n)
    for (int st = 0; st < 5; ++st) {
      if ((rc = launch(c, true, cur, nxt, res, kRkA[st], kRkB[st], dt, t0 + (n + kRkC[st]) * dt, s))) return rc;
      std::swap(cur, nxt);
    }
  if (cur != q) {
    hipError_t e = hipMemcpyAsync(q, cur, (size_t)4 * c->K * c->Np * c->rsz, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(BBWADG_EHIP, "state copy: %s", hipGetErrorString(e));
  }
  return 0;
}

int bbwadg_suggest_dt(const bbwadg_ctx* c, double cfl, double* dt) {
  if (!c || !dt) return fail(BBWADG_EINVAL, "NULL argument");
  if (!(cfl > 0)) return fail(BBWADG_EINVAL, "cfl must be > 0");
  if (!c->c2_set) return fail(BBWADG_EC2, "c^2 not set");
  double c2max = 0, fmax = 0;
  for (double v : c->c2) c2max = std::max(c2max, v);
  for (double v : c->fscale) fmax = std::max(fmax, v);
  double CN = (c->N + 1.0) * (c->N + 3.0) / 3.0;
  *dt = cfl / (std::sqrt(c2max) * CN * fmax);
  return 0;
}

int bbwadg_l2norm2(bbwadg_ctx* c, const void* q, double out[4], void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !out) return fail(BBWADG_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  int e = launch_l2norm(c->N, c->dtype, q, c->K, (const double*)c->d_J, (const double*)c->d_mass,
                        (double*)c->d_partial, c->nred_blocks, s);
  if (e) return fail(BBWADG_EHIP, "l2norm launch: %s", hipGetErrorString((hipError_t)e));
  std::vector<double> part((size_t)c->nred_blocks * 4);
  hipError_t he = hipMemcpyAsync(part.data(), c->d_partial, part.size() * 8, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return fail(BBWADG_EHIP, "l2norm copy: %s", hipGetErrorString(he));
  for (int f = 0; f < 4; ++f) {
    double acc = 0;
    for (int b = 0; b < c->nred_blocks; ++b) acc += part[(size_t)b * 4 + f];
    out[f] = acc;
  }
  return 0;
}

int bbwadg_l2norm2_noalloc(bbwadg_ctx* c, const void* q, double* out, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !out) return fail(BBWADG_EINVAL, "NULL argument");
  if (c->nred_blocks > kScratchBlocks)
    return fail(BBWADG_EINVAL, "%d reduction blocks exceed the fixed scratch of %d", c->nred_blocks, kScratchBlocks);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return fail(BBWADG_EINVAL, "the current device is not the context's device %d", c->device);
  const int e = l2norm2_noalloc(c->N, c->dtype, q, c->K, (const double*)c->d_J, (const double*)c->d_mass,
                                c->nred_blocks, out, stream);
  if (e) return fail(BBWADG_EHIP, "l2norm (no allocation) launch: %s", hipGetErrorString((hipError_t)e));
  return 0;
}

int bbwadg_l2error2(bbwadg_ctx* c, const void* q, int64_t k0, int64_t k1, const double* exact, double out[4],
                    void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !exact || !out) return fail(BBWADG_EINVAL, "NULL argument");
  return quad_reduce(c, 0, q, k0, k1, exact, out, (hipStream_t)stream);
}

int bbwadg_energy(bbwadg_ctx* c, const void* q, int64_t k0, int64_t k1, double out[4], void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !out) return fail(BBWADG_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = sync_c2(c, s))) return rc;
  return quad_reduce(c, 1, q, k0, k1, nullptr, out, s);
}

int bbwadg_project_fn(bbwadg_ctx* c, double (*fn)(double, double, double, void*), void* user, int32_t field,
                      void* q_out, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!fn || !q_out) return fail(BBWADG_EINVAL, "NULL argument");
  if (field < 0 || field > 3) return fail(BBWADG_EINVAL, "field %d outside [0,3]", field);
  const Projector& pr = get_projector(c, c->N);
  const int64_t K = c->K;
  const int np = c->Np;
  std::vector<double> coef((size_t)K * np);
  const int64_t chunk = 4096;
  std::vector<double> xyz, smp;
  for (int64_t k0 = 0; k0 < K; k0 += chunk) {
    int64_t k1 = std::min(K, k0 + chunk);
    xyz.resize((size_t)(k1 - k0) * pr.nq * 3);
    smp.resize((size_t)(k1 - k0) * pr.nq);
    if ((rc = bbwadg_projection_points(c, c->N, k0, k1, xyz.data()))) return rc;
    for (size_t i = 0; i < smp.size(); ++i) {
      smp[i] = fn(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], user);
      if (!std::isfinite(smp[i])) return fail(BBWADG_EINVAL, "non-finite sample in element %lld", (long long)(k0 + (int64_t)i / pr.nq));
    }
    if ((rc = bbwadg_project_samples(c, c->N, k0, k1, smp.data(), &coef[(size_t)k0 * np]))) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  char* dst = (char*)q_out + (size_t)field * K * np * c->rsz;
  std::vector<float> f32;
  const void* src = coef.data();
  size_t bytes = coef.size() * 8;
  if (c->dtype == BBWADG_F32) {
    f32 = convert<float>(coef);
    src = f32.data();
    bytes = f32.size() * 4;
  }
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // src is a local buffer
  if (e != hipSuccess) return fail(BBWADG_EHIP, "state upload: %s", hipGetErrorString(e));
  return 0;
}

int bbwadg_dense_npoints(const bbwadg_ctx* c, int64_t* nq) {
  if (!c || !nq) return fail(BBWADG_EINVAL, "NULL argument");
  const int64_t n = dense_rule_n(c);
  *nq = n * n * n;
  return 0;
}

int bbwadg_dense_points(const bbwadg_ctx* ctx, int64_t k0, int64_t k1, double* xyz_out) {
  if (!ctx || !xyz_out) return fail(BBWADG_EINVAL, "NULL argument");
  if (k0 < 0 || k1 > ctx->K || k0 > k1) return fail(BBWADG_EINVAL, "bad element range");
  auto* c = const_cast<bbwadg_ctx*>(ctx);
  const Projector& pr = get_dense(c);
  for (int64_t k = k0; k < k1; ++k) {
    const int32_t* v = &c->etov[4 * k];
    for (int q = 0; q < pr.nq; ++q)
      for (int d = 0; d < 3; ++d) {
        ld x = 0;
        for (int j = 0; j < 4; ++j) x += pr.lam[q][j] * (ld)c->xyz[3 * (size_t)v[j] + d];
        xyz_out[((size_t)(k - k0) * pr.nq + q) * 3 + d] = (double)x;
      }
  }
  return 0;
}

int bbwadg_dense_set_c2(bbwadg_ctx* c, const double* c2q, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!c2q && !c->c2_set) return fail(BBWADG_EC2, "c^2 not set (pass point values or set c^2_M first)");
  if ((rc = dense_tables(c))) return rc;
  const Projector& pr = c->dense;
  const int64_t K = c->K;
  const int nq = pr.nq, nqp = c->dense_nqp, mp = c->Mp;
  std::vector<double> buf((size_t)K * nqp, 0.0);
  std::vector<ld> bm;
  if (!c2q) {  // c^2_M at the dense points
    auto AM = mi3_list(c->M);
    bm.resize((size_t)nq * mp);
    for (int q = 0; q < nq; ++q)
      for (int b = 0; b < mp; ++b) bm[(size_t)q * mp + b] = bernstein(c->M, AM[b], pr.lam[q]);
  }
  std::atomic<int> bad{0};
  parallel_for(0, K, [&](int64_t a, int64_t b) {
    for (int64_t k = a; k < b; ++k)
      for (int q = 0; q < nq; ++q) {
        double v;
        if (c2q) {
          v = c2q[(size_t)k * nq + q];
        } else {
          ld acc = 0;
          for (int j = 0; j < mp; ++j) acc += bm[(size_t)q * mp + j] * (ld)c->c2[(size_t)k * mp + j];
          v = (double)acc;
        }
        if (!std::isfinite(v) || !(v > 0)) bad.store(1, std::memory_order_relaxed);
        buf[(size_t)k * nqp + q] = v;
      }
  });
  if (bad.load()) return fail(BBWADG_EC2, "c^2 at the dense points must be finite and positive");
  if (!c->d_c2q && (rc = dmalloc(&c->d_c2q, buf.size() * c->rsz))) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::vector<float> buf32;
  if (c->dtype == BBWADG_F32) buf32 = convert<float>(buf);
  const void* src = c->dtype == BBWADG_F32 ? (const void*)buf32.data() : (const void*)buf.data();
  hipError_t e = hipMemcpyAsync(c->d_c2q, src, buf.size() * c->rsz, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // buf is a local buffer
  if (e != hipSuccess) return fail(BBWADG_EHIP, "c^2 point values upload: %s", hipGetErrorString(e));
  c->c2q_set = true;
  return 0;
}

int bbwadg_dense_update(bbwadg_ctx* c, const void* r, void* out, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!r || !out) return fail(BBWADG_EINVAL, "NULL argument");
  if (!c->c2q_set) return fail(BBWADG_EC2, "call bbwadg_dense_set_c2 first");
  int e;
  if (c->dtype == BBWADG_F64) {
    DenseArgs<double> a{};
    a.r = (const double*)r;
    a.out = (double*)out;
    a.va = (const double*)c->d_dva;
    a.pa = (const double*)c->d_dpa;
    a.c2q = (const double*)c->d_c2q;
    a.K = c->K;
    a.nqp = c->dense_nqp;
    a.nqc = c->dense_nqp / 16;
    e = launch_wadg_dense<double>(c->N, a, stream);
  } else {
    DenseArgs<float> a{};
    a.r = (const float*)r;
    a.out = (float*)out;
    a.va = (const float*)c->d_dva32;
    a.pa = (const float*)c->d_dpa32;
    a.c2q = (const float*)c->d_c2q;
    a.K = c->K;
    a.nqp = c->dense_nqp;
    a.nqc = c->dense_nqp / 16;
    e = launch_wadg_dense<float>(c->N, a, stream);
  }
  if (e) return fail(BBWADG_EHIP, "dense update launch: %s", hipGetErrorString((hipError_t)e));
  return 0;
}

int bbwadg_rhs_dense(bbwadg_ctx* c, const void* q, void* rhs, double t, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !rhs) return fail(BBWADG_EINVAL, "NULL state pointer");
  if (q == rhs) return fail(BBWADG_EINVAL, "q and rhs must not overlap");
  if (!c->c2q_set) return fail(BBWADG_EC2, "call bbwadg_dense_set_c2 first");
  hipStream_t s = (hipStream_t)stream;
  int e;
  if (c->dtype == BBWADG_F64) {
    StageArgs<double> a = make_args<double>(c);  // the plain DG right-hand side: c^2 = 1, M = 0
    a.c2 = (const double*)c->d_ones;
    a.src_amp = source_factor(c, t);
    a.qin = (const double*)q;
    a.qout = (double*)rhs;
    e = launch_stage_f64(c->N, 0, false, a, s);
  } else {
    StageArgs<float> a = make_args<float>(c);
    a.c2 = (const float*)c->d_ones;
    a.src_amp = (float)source_factor(c, t);
    a.qin = (const float*)q;
    a.qout = (float*)rhs;
    e = launch_stage_f32(c->N, 0, false, a, s);
  }
  if (e) return fail(BBWADG_EHIP, "stage launch: %s", hipGetErrorString((hipError_t)e));
  return bbwadg_dense_update(c, rhs, rhs, stream);  // the p field, in place
}

int bbwadg_set_source(bbwadg_ctx* c, const double* g, double amp, double omega, double phase) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!g) {  // clear
    if (c->d_src) {
      (void)hipDeviceSynchronize();
      (void)hipFree(c->d_src);
      c->d_src = nullptr;
    }
    return 0;
  }
  if (!std::isfinite(amp) || !std::isfinite(omega) || !std::isfinite(phase))
    return fail(BBWADG_EINVAL, "source time factor must be finite");
  const size_t n = (size_t)c->K * c->Np;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(g[i])) return fail(BBWADG_EINVAL, "source coefficient %zu not finite", i);
  if (!c->d_src && (rc = dmalloc(&c->d_src, n * c->rsz))) return rc;
  if (c->dtype == BBWADG_F64) {
    rc = upload(c->d_src, g, n * 8);
  } else {
    std::vector<float> f(g, g + n);
    rc = upload(c->d_src, f.data(), n * 4);
  }
  if (rc) return rc;
  c->src_amp = amp;
  c->src_omega = omega;
  c->src_phase = phase;
  return 0;
}

int32_t bbwadg_coef_index(int32_t a1, int32_t a2, int32_t a3) {
  if (a1 < 0 || a2 < 0 || a3 < 0) return fail(BBWADG_EINVAL, "negative multi-index entry");
  const int s = a1 + a2 + a3;
  if (s > kMaxDeg) return fail(BBWADG_EINVAL, "degree %d above %d", s, kMaxDeg);
  return dimp(s - 1) + a3 * (2 * s + 3 - a3) / 2 + a2;
}

}  // extern "C"

// ------------------------------------------------------------ receivers and the adjoint
namespace {

// b <- A^{-1} b for the symmetric positive definite A [n][n] (long-double Cholesky).
void spd_solve(std::vector<ld> A, int n, std::vector<ld>& b) {
  for (int j = 0; j < n; ++j) {
    ld s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    const ld d = std::sqrt(s);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      ld t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / d;
    }
  }
  for (int i = 0; i < n; ++i) {
    ld t = b[i];
    for (int k = 0; k < i; ++k) t -= A[(size_t)i * n + k] * b[k];
    b[i] = t / A[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    ld t = b[i];
    for (int k = i + 1; k < n; ++k) t -= A[(size_t)k * n + i] * b[k];
    b[i] = t / A[(size_t)i * n + i];
  }
}

inline int launch_typed(int N, int M, bool update, const StageArgs<double>& a, hipStream_t s) {
  return launch_stage_f64(N, M, update, a, s);
}
inline int launch_typed(int N, int M, bool update, const StageArgs<float>& a, hipStream_t s) {
  return launch_stage_f32(N, M, update, a, s);
}

// One stage-kernel launch with the weight, source and degree M chosen by the caller: the
// plain DG operator is M = 0 with c^2 = 1; the weight adjustment alone is a zero state with
// the input passed as the source (amplitude 1), since the kernel adds the source to r_p
// before the weight-adjusted projection.
template <typename real>
int stage_custom(bbwadg_ctx* c, int M, const void* c2, const void* src, double amp, bool update, const void* qin,
                 void* qout, void* res, double ra, double rb, double dt, hipStream_t s) {
  StageArgs<real> a = make_args<real>(c);
  a.c2 = (const real*)c2;
  a.src = (const real*)src;
  a.src_amp = (real)amp;
  a.qin = (const real*)qin;
  a.qout = (real*)qout;
  a.res = (real*)res;
  a.rk_a = (real)ra;
  a.rk_b = (real)rb;
  a.dt = (real)dt;
  const int e = launch_typed(c->N, M, update, a, s);
  if (e) return fail(BBWADG_EHIP, "stage launch: %s", hipGetErrorString((hipError_t)e));
  return 0;
}

int hip_check(hipError_t e, const char* what) {
  return e == hipSuccess ? 0 : fail(BBWADG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Device buffers of one call, freed together (after the caller's stream has drained).
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    if (!ptrs.empty()) (void)hipDeviceSynchronize();  // also on error paths, with work in flight
    for (void* p : ptrs) (void)hipFree(p);
  }
  int get(void** p, size_t bytes) {
    int rc = dmalloc(p, bytes ? bytes : 8);
    if (!rc) ptrs.push_back(*p);
    return rc;
  }
};

// The plain-DG weight (ones) and the gradient's rule tables, built on first use.
int adjoint_setup(bbwadg_ctx* c) {
  int rc;
  if (!c->d_adj_ones) {
    if (c->dtype == BBWADG_F64) {
      std::vector<double> ones((size_t)c->K, 1.0);
      if ((rc = dmalloc(&c->d_adj_ones, ones.size() * 8)) || (rc = upload(c->d_adj_ones, ones.data(), ones.size() * 8)))
        return rc;
    } else {
      std::vector<float> ones((size_t)c->K, 1.0f);
      if ((rc = dmalloc(&c->d_adj_ones, ones.size() * 4)) || (rc = upload(c->d_adj_ones, ones.data(), ones.size() * 4)))
        return rc;
    }
  }
  if (!c->d_adj_bwa) {
    // V_q of the dense rule (exact to degree 2N + M) is shared with the dense WADG baseline
    if ((rc = dense_tables(c))) return rc;
    Projector pm;
    build_projector_rule(c->M, dense_rule_n(c), pm);
    const int nq = pm.nq, Mp = c->Mp, nqc = c->dense_nqp / 16;
    std::vector<double> bwa((size_t)nqc * 4 * 64, 0.0);
    for (int qc = 0; qc < nqc; ++qc)
      for (int ks = 0; ks < 4; ++ks)
        for (int l = 0; l < 64; ++l) {
          const int g = l % 16, q = 16 * qc + 4 * ks + l / 16;
          if (g < Mp && q < nq) bwa[((size_t)qc * 4 + ks) * 64 + l] = pm.w[q] * pm.B[(size_t)q * Mp + g];
        }
    if ((rc = dmalloc(&c->d_adj_bwa, bwa.size() * 8)) || (rc = upload(c->d_adj_bwa, bwa.data(), bwa.size() * 8)))
      return rc;
  }
  return 0;
}

// out = Pi_N(c^2_M x) for one field (the update kernel on its own).
template <typename real>
int wadg_apply(bbwadg_ctx* c, const void* x, void* out, hipStream_t s) {
  ElasticArgs<real> a{};
  a.r = (const real*)x;
  a.out = (real*)out;
  a.rho_inv = (const real*)c->d_c2;
  a.K = c->K;
  set_cj(c, a);
  const int e = launch_wadg_update<real>(c->N, c->M, a, s);
  return e ? fail(BBWADG_EHIP, "update launch: %s", hipGetErrorString((hipError_t)e)) : 0;
}

template <typename real>
int misfit_gradient_typed(bbwadg_ctx* c, const void* q0, double t0, double dt, int32_t nsteps, const double* data,
                          int32_t ckpt, double* traces, double* misfit, double* grad, hipStream_t s) {
  int rc;
  const int64_t K = c->K;
  const int Np = c->Np, nrec = c->nrec;
  const size_t n1 = (size_t)K * Np, n4 = 4 * n1, rb = sizeof(real);
  const int C = std::min(ckpt, nsteps), nseg = (nsteps + C - 1) / C;
  Scratch ws;
  void *qa, *qb, *res, *ck, *tr = traces, *resid;
  if ((rc = ws.get(&qa, n4 * rb)) || (rc = ws.get(&qb, n4 * rb)) || (rc = ws.get(&res, n4 * rb)) ||
      (rc = ws.get(&ck, (size_t)nseg * n4 * rb)) || (rc = ws.get(&resid, (size_t)nsteps * nrec * 8)))
    return rc;
  if (!tr && (rc = ws.get(&tr, (size_t)nsteps * nrec * 8))) return rc;
  if ((rc = hip_check(hipMemsetAsync(res, 0, n4 * rb, s), "memset")) ||
      (rc = hip_check(hipMemcpyAsync(qa, q0, n4 * rb, hipMemcpyDeviceToDevice, s), "copy q0")))
    return rc;
  const int32_t* elem = (const int32_t*)c->d_rec_elem;
  const double* rbasis = (const double*)c->d_rec_basis;
  // forward: checkpoints at the start of every segment, receivers after every step
  void* cur = qa;
  void* nxt = qb;
  for (int32_t n = 0; n < nsteps; ++n) {
    if (n % C == 0 &&
        (rc = hip_check(hipMemcpyAsync((char*)ck + (size_t)(n / C) * n4 * rb, cur, n4 * rb, hipMemcpyDeviceToDevice, s),
                        "checkpoint")))
      return rc;
    for (int st = 0; st < 5; ++st) {
      if ((rc = launch(c, true, cur, nxt, res, kRkA[st], kRkB[st], dt, t0 + (n + kRkC[st]) * dt, s))) return rc;
      std::swap(cur, nxt);
    }
    int e = launch_sample<real>((const real*)cur, elem, rbasis, nrec, Np, (double*)tr + (size_t)n * nrec, s);
    if (e) return fail(BBWADG_EHIP, "receiver sample: %s", hipGetErrorString((hipError_t)e));
  }
  // misfit and residuals on the host (FP64)
  const size_t nt = (size_t)nsteps * nrec;
  std::vector<double> htr(nt), hd(nt, 0.0);
  if ((rc = hip_check(hipMemcpyAsync(htr.data(), tr, nt * 8, hipMemcpyDeviceToHost, s), "traces download")))
    return rc;
  if (data && (rc = hip_check(hipMemcpyAsync(hd.data(), data, nt * 8, hipMemcpyDeviceToHost, s), "data download")))
    return rc;
  if ((rc = hip_check(hipStreamSynchronize(s), "sync"))) return rc;
  double J = 0.0;
  for (size_t i = 0; i < nt; ++i) {
    if (!std::isfinite(hd[i])) return fail(BBWADG_EINVAL, "data value %zu not finite", i);
    hd[i] = htr[i] - hd[i];
    J += 0.5 * hd[i] * hd[i];
  }
  *misfit = J;
  if (!grad) return hip_check(hipStreamSynchronize(s), "sync");
  if ((rc = hip_check(hipMemcpyAsync(resid, hd.data(), nt * 8, hipMemcpyHostToDevice, s), "residual upload")) ||
      (rc = adjoint_setup(c)))
    return rc;
  // backward in the variables z = (M S)^{-1} lambda: per reversed stage
  //   v = z_r + b_k z_q;  grad += dt dW/dc(y_k, v);  z_q += dt B W v;  z_r = a_k v
  void *ys, *zq, *v, *w4, *t4;
  if ((rc = ws.get(&ys, (size_t)C * 5 * n1 * rb)) || (rc = ws.get(&zq, n4 * rb)) || (rc = ws.get(&v, n4 * rb)) ||
      (rc = ws.get(&w4, n4 * rb)) || (rc = ws.get(&t4, n4 * rb)))
    return rc;
  if ((rc = hip_check(hipMemsetAsync(zq, 0, n4 * rb, s), "memset")) ||
      (rc = hip_check(hipMemsetAsync(v, 0, n4 * rb, s), "memset")) ||
      (rc = hip_check(hipMemsetAsync(grad, 0, (size_t)K * c->Mp * 8, s), "memset")))
    return rc;
  C2GradArgs<real> ga{};
  ga.va = (const double*)c->d_dva;
  ga.bwa = (const double*)c->d_adj_bwa;
  ga.J = (const double*)c->d_J;
  ga.grad = grad;
  ga.scale = dt;
  ga.K = K;
  ga.Mp = c->Mp;
  ga.nqc = c->dense_nqp / 16;
  ga.v = (const real*)v;
  const void* ones = c->d_adj_ones;
  int e;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int32_t na = seg * C, nb = std::min(nsteps, na + C);
    // recompute the segment, keeping y = (B q)_p of every stage input (source included): the
    // update launches write it through StageArgs::rp_out
    if ((rc = hip_check(hipMemcpyAsync(qa, (char*)ck + (size_t)seg * n4 * rb, n4 * rb, hipMemcpyDeviceToDevice, s),
                        "restore")))
      return rc;
    cur = qa;
    nxt = qb;
    for (int32_t n = na; n < nb; ++n)
      for (int st = 0; st < 5; ++st) {
        const double ts = t0 + (n + kRkC[st]) * dt;
        // the update launch also writes y = (B q)_p of its input (source included) to the slot
        void* yslot = (char*)ys + ((size_t)(n - na) * 5 + st) * n1 * rb;
        if ((rc = launch(c, true, cur, nxt, res, kRkA[st], kRkB[st], dt, ts, s, yslot))) return rc;
        std::swap(cur, nxt);
      }
    for (int32_t n = nb - 1; n >= na; --n) {
      // dJ/dq after step n, then v = z_r + b_5 z_q with z_r = a_1 v = 0
      if ((e = launch_inject<real>((real*)zq, elem, (const double*)c->d_rec_kvec, (const double*)resid + (size_t)n * nrec,
                                   nrec, Np, s)) ||
          (e = launch_lincomb<real>((real*)v, (const real*)zq, 0.0, kRkB[4], (int64_t)n4, s)))
        return fail(BBWADG_EHIP, "adjoint bookkeeping: %s", hipGetErrorString((hipError_t)e));
      for (int st = 4; st >= 0; --st) {
        ga.y = (const real*)((char*)ys + ((size_t)(n - na) * 5 + st) * n1 * rb);
        if ((e = launch_c2grad<real>(c->N, ga, s))) return fail(BBWADG_EHIP, "c2 gradient: %s", hipGetErrorString((hipError_t)e));
        // w4 = (W v_p, v_u), t4 = B w4
        if ((rc = wadg_apply<real>(c, v, w4, s)) ||
            (rc = hip_check(hipMemcpyAsync((char*)w4 + n1 * rb, (char*)v + n1 * rb, 3 * n1 * rb, hipMemcpyDeviceToDevice, s),
                            "copy u")) ||
            (rc = stage_custom<real>(c, 0, ones, nullptr, 0.0, false, w4, t4, nullptr, 0, 0, 0, s)))
          return rc;
        // z_q += dt t4; for the next reversed stage v = z_r + b_{k-1} z_q with z_r = a_k v
        if ((e = launch_back_update<real>((real*)zq, (real*)v, (const real*)t4, dt, kRkA[st], st > 0 ? kRkB[st - 1] : 0.0,
                                          st > 0, (int64_t)n4, s)))
          return fail(BBWADG_EHIP, "adjoint bookkeeping: %s", hipGetErrorString((hipError_t)e));
      }
    }
  }
  return hip_check(hipStreamSynchronize(s), "sync");
}

}  // namespace

extern "C" {

int bbwadg_set_receivers(bbwadg_ctx* c, int32_t nrec, const double* xyz) {
  if (!c) return fail(BBWADG_EINVAL, "NULL context");
  if (nrec < 0 || (nrec > 0 && !xyz)) return fail(BBWADG_EINVAL, "bad receiver count or NULL coordinates");
  if (nrec > (1 << 20)) return fail(BBWADG_EINVAL, "too many receivers");
  const int Np = c->Np;
  std::vector<int32_t> elem(nrec, -1);
  std::vector<double> basis((size_t)nrec * Np), kvec((size_t)nrec * Np);
  auto A = mi3_list(c->N);
  std::vector<ld> Mm = bernstein_mass(c->N);
  for (int32_t r = 0; r < nrec; ++r) {
    const double* x = xyz + 3 * (size_t)r;
    if (!std::isfinite(x[0]) || !std::isfinite(x[1]) || !std::isfinite(x[2]))
      return fail(BBWADG_EINVAL, "receiver %d not finite", r);
    std::array<ld, 4> lam{};
    for (int64_t k = 0; k < c->K && elem[r] < 0; ++k) {  // the lowest-numbered containing element
      const double* v0 = &c->xyz[3 * (size_t)c->etov[4 * k]];
      ld l[4];
      ld sum = 0;
      for (int j = 0; j < 3; ++j) {
        ld t = 0;
        for (int i = 0; i < 3; ++i) t += (ld)c->G[9 * k + 3 * i + j] * ((ld)x[i] - v0[i]);
        l[j + 1] = t / 2;  // (r_j + 1) / 2
        sum += l[j + 1];
      }
      l[0] = 1 - sum;
      if (l[0] >= -1e-10L && l[1] >= -1e-10L && l[2] >= -1e-10L && l[3] >= -1e-10L) {
        elem[r] = (int32_t)k;
        for (int j = 0; j < 4; ++j) lam[j] = l[j];
      }
    }
    if (elem[r] < 0) return fail(BBWADG_EINVAL, "receiver %d (%g, %g, %g) is outside the mesh", r, x[0], x[1], x[2]);
    std::vector<ld> b(Np);
    for (int i = 0; i < Np; ++i) b[i] = bernstein(c->N, A[i], lam);
    for (int i = 0; i < Np; ++i) basis[(size_t)r * Np + i] = (double)b[i];
    spd_solve(Mm, Np, b);
    for (int i = 0; i < Np; ++i) kvec[(size_t)r * Np + i] = (double)(b[i] / c->J[elem[r]]);
  }
  c->rec_elem = elem;
  c->rec_basis = basis;
  c->rec_kvec = kvec;
  c->nrec = nrec;
  if (c->mode != BBWADG_DEVICE || nrec == 0) return 0;
  int rc;
  for (void** p : {&c->d_rec_elem, &c->d_rec_basis, &c->d_rec_kvec})
    if (*p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(*p);
      *p = nullptr;
    }
  if ((rc = dmalloc(&c->d_rec_elem, (size_t)nrec * 4)) || (rc = upload(c->d_rec_elem, elem.data(), (size_t)nrec * 4)) ||
      (rc = dmalloc(&c->d_rec_basis, basis.size() * 8)) || (rc = upload(c->d_rec_basis, basis.data(), basis.size() * 8)) ||
      (rc = dmalloc(&c->d_rec_kvec, kvec.size() * 8)) || (rc = upload(c->d_rec_kvec, kvec.data(), kvec.size() * 8)))
    return rc;
  return 0;
}

int bbwadg_receiver_elements(const bbwadg_ctx* c, int32_t* elem_out) {
  if (!c || !elem_out) return fail(BBWADG_EINVAL, "NULL argument");
  std::copy(c->rec_elem.begin(), c->rec_elem.end(), elem_out);
  return 0;
}

int bbwadg_misfit_gradient(bbwadg_ctx* c, const void* q0, double t0, double dt, int32_t nsteps, const double* data,
                           int32_t checkpoint_every, double* traces, double* misfit, double* grad, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q0 || !misfit) return fail(BBWADG_EINVAL, "NULL q0 or misfit");
  if (c->nrec <= 0) return fail(BBWADG_EINVAL, "no receivers (call bbwadg_set_receivers)");
  if (nsteps < 1 || checkpoint_every < 1 || !std::isfinite(dt) || !std::isfinite(t0))
    return fail(BBWADG_EINVAL, "bad nsteps, checkpoint interval, dt or t0");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = sync_c2(c, s))) return rc;
  if (c->dtype == BBWADG_F64)
    return misfit_gradient_typed<double>(c, q0, t0, dt, nsteps, data, checkpoint_every, traces, misfit, grad, s);
  return misfit_gradient_typed<float>(c, q0, t0, dt, nsteps, data, checkpoint_every, traces, misfit, grad, s);
}

}  // extern "C"

namespace {

// Face coefficient m of face f <-> face multi-index (b0, b1, b2) on the face's vertices in
// ascending local order, m = s(s+1)/2 + b2 with s = b1 + b2: the volume position of that
// coefficient (alpha_f = 0).
int elastic_tables(bbwadg_ctx* c) {
  if (c->d_el_fpos) return 0;
  const int N = c->N, Nfp = c->Nfp;
  std::vector<int32_t> fpos(4 * Nfp);
  for (int f = 0; f < 4; ++f) {
    int vs[3], n = 0;
    for (int v = 0; v < 4; ++v)
      if (v != f) vs[n++] = v;
    for (int s = 0; s <= N; ++s)
      for (int b2 = 0; b2 <= s; ++b2) {
        const int b[3] = {N - s, s - b2, b2};
        int al[4] = {0, 0, 0, 0};
        for (int q = 0; q < 3; ++q) al[vs[q]] = b[q];
        const int d = al[1] + al[2] + al[3];
        fpos[f * Nfp + s * (s + 1) / 2 + b2] = dimp(d - 1) + al[3] * (2 * d + 3 - al[3]) / 2 + al[2];
      }
  }
  void* p = nullptr;
  int rc;
  if ((rc = dmalloc(&p, fpos.size() * 4))) return rc;
  if ((rc = upload(p, fpos.data(), fpos.size() * 4))) {
    (void)hipFree(p);
    return rc;
  }
  c->d_el_fpos = p;
  return 0;
}

template <typename real>
int elastic_update_typed(bbwadg_ctx* c, const void* r, void* out, void* res, void* q, double ra, double rb, double dt,
                         void* stream) {
  ElasticArgs<real> a{};
  a.r = (const real*)r;
  a.out = (real*)out;
  a.rho_inv = (const real*)c->d_el_rho;
  a.lam = (const real*)c->d_el_lam;
  a.mu = (const real*)c->d_el_mu;
  a.K = c->K;
  set_cj(c, a);
  a.res = (real*)res;
  a.q = (real*)q;
  a.rk_a = (real)ra;
  a.rk_b = (real)rb;
  a.dt = (real)dt;
  return launch_elastic_update<real>(c->N, c->M, a, stream);
}

// The elastic update of r into out, or (res != nullptr) a low-storage RK stage from it.
int elastic_update_launch(bbwadg_ctx* c, const void* r, void* out, void* res, void* q, double ra, double rb,
                          double dt, void* stream) {
  const int e = c->dtype == BBWADG_F64 ? elastic_update_typed<double>(c, r, out, res, q, ra, rb, dt, stream)
                                       : elastic_update_typed<float>(c, r, out, res, q, ra, rb, dt, stream);
  return e ? fail(BBWADG_EHIP, "elastic update launch: %s", hipGetErrorString((hipError_t)e)) : 0;
}

template <typename real>
int elastic_rhs_typed(bbwadg_ctx* c, const void* q, void* out, int32_t wall, double tau_v, double tau_s, hipStream_t s) {
  ElasticRhsArgs<real> a{};
  a.q = (const real*)q;
  a.out = (real*)out;
  a.geo = (const real*)c->d_geo;
  a.conn = (const int32_t*)c->d_conn;
  a.fpos = (const int32_t*)c->d_el_fpos;
  a.K = c->K;
  a.tau_v = (real)tau_v;
  a.tau_s = (real)tau_s;
  a.wall = wall;
  const int e = launch_elastic_rhs<real>(c->N, a, s);
  return e ? fail(BBWADG_EHIP, "elastic right-hand side launch: %s", hipGetErrorString((hipError_t)e)) : 0;
}

}  // namespace

extern "C" {

int bbwadg_elastic_rhs(bbwadg_ctx* c, const void* q, void* rhs, int32_t wall, double tau_v, double tau_s,
                       int32_t weighted, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !rhs) return fail(BBWADG_EINVAL, "NULL state pointer");
  if (q == rhs) return fail(BBWADG_EINVAL, "q and rhs must not overlap");
  if (wall != 0 && wall != 1) return fail(BBWADG_EINVAL, "wall must be 0 (traction-free) or 1 (rigid)");
  if (!(tau_v >= 0) || !(tau_s >= 0) || !std::isfinite(tau_v) || !std::isfinite(tau_s))
    return fail(BBWADG_EINVAL, "tau must be finite and >= 0");
  if (weighted && !c->d_el_rho) return fail(BBWADG_EC2, "elastic media not set (call bbwadg_elastic_set_media)");
  if ((rc = elastic_tables(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  void* dst = rhs;
  if (weighted) {
    if (!c->d_el_tmp && (rc = dmalloc(&c->d_el_tmp, (size_t)9 * c->K * c->Np * c->rsz))) return rc;
    dst = c->d_el_tmp;
  }
  rc = c->dtype == BBWADG_F64 ? elastic_rhs_typed<double>(c, q, dst, wall, tau_v, tau_s, s)
                              : elastic_rhs_typed<float>(c, q, dst, wall, tau_v, tau_s, s);
  if (rc || !weighted) return rc;
  return bbwadg_elastic_update(c, dst, rhs, stream);
}

int bbwadg_elastic_step(bbwadg_ctx* c, void* q, void* res, double dt, int32_t nsteps, int32_t wall, double tau_v,
                        double tau_s, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!q || !res) return fail(BBWADG_EINVAL, "NULL state pointer");
  if (q == res) return fail(BBWADG_EINVAL, "q and res must not overlap");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(BBWADG_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(BBWADG_EINVAL, "nsteps must be >= 0");
  if (!c->d_el_rho) return fail(BBWADG_EC2, "elastic media not set (call bbwadg_elastic_set_media)");
  const int64_t n = (int64_t)9 * c->K * c->Np;
  // The RK bookkeeping rides on the update's final write for N <= 7; above, at the update's
  // low occupancy, the extra read-modify-write is exposed (measured slower at N = 9) and the
  // update writes Pi(r) for two lincomb passes instead.
  const bool fused = c->N <= 7;
  if (!c->d_el_tmp && (rc = dmalloc(&c->d_el_tmp, (size_t)n * c->rsz))) return rc;
  if (!fused && !c->d_el_rhs && (rc = dmalloc(&c->d_el_rhs, (size_t)n * c->rsz))) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int32_t it = 0; it < nsteps; ++it)
    for (int st = 0; st < 5; ++st) {
      // r = the right-hand side of q; res = a_k res + dt Pi(r), q = q + b_k res
      if ((rc = bbwadg_elastic_rhs(c, q, c->d_el_tmp, wall, tau_v, tau_s, 0, stream))) return rc;
      if (fused) {
        if ((rc = elastic_update_launch(c, c->d_el_tmp, nullptr, res, q, kRkA[st], kRkB[st], dt, stream))) return rc;
        continue;
      }
      if ((rc = elastic_update_launch(c, c->d_el_tmp, c->d_el_rhs, nullptr, nullptr, 0.0, 0.0, 0.0, stream))) return rc;
      int e = c->dtype == BBWADG_F64
                  ? launch_lincomb<double>((double*)res, (const double*)c->d_el_rhs, kRkA[st], dt, n, s)
                  : launch_lincomb<float>((float*)res, (const float*)c->d_el_rhs, kRkA[st], dt, n, s);
      if (!e)
        e = c->dtype == BBWADG_F64 ? launch_lincomb<double>((double*)q, (const double*)res, 1.0, kRkB[st], n, s)
                                   : launch_lincomb<float>((float*)q, (const float*)res, 1.0, kRkB[st], n, s);
      if (e) return fail(BBWADG_EHIP, "elastic step update: %s", hipGetErrorString((hipError_t)e));
    }
  return 0;
}

int bbwadg_wadg_update(bbwadg_ctx* c, const void* r, void* out, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!r || !out) return fail(BBWADG_EINVAL, "NULL argument");
  if (r == out) return fail(BBWADG_EINVAL, "r and out must not overlap");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = sync_c2(c, s))) return rc;
  int e;
  if (c->dtype == BBWADG_F64) {
    ElasticArgs<double> a{};
    a.r = (const double*)r;
    a.out = (double*)out;
    a.rho_inv = (const double*)c->d_c2;
    a.K = c->K;
    set_cj(c, a);
    e = launch_wadg_update<double>(c->N, c->M, a, s);
  } else {
    ElasticArgs<float> a{};
    a.r = (const float*)r;
    a.out = (float*)out;
    a.rho_inv = (const float*)c->d_c2;
    a.K = c->K;
    set_cj(c, a);
    e = launch_wadg_update<float>(c->N, c->M, a, s);
  }
  if (e) return fail(BBWADG_EHIP, "update launch: %s", hipGetErrorString((hipError_t)e));
  return 0;
}

int bbwadg_elastic_set_media(bbwadg_ctx* c, const double* rho_inv, const double* lam, const double* mu) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!rho_inv || !lam || !mu) return fail(BBWADG_EINVAL, "NULL medium array");
  const size_t n = (size_t)c->K * c->Mp;
  const double* src[3] = {rho_inv, lam, mu};
  // The weights of the velocity-stress mass matrices must be positive everywhere: 1/rho,
  // mu and the bulk term 3 lambda + 2 mu (a degree-M polynomial with coefficients
  // 3 lambda_b + 2 mu_b). Everything is checked before anything is uploaded.
  std::vector<double> bulk(n);
  for (size_t i = 0; i < n; ++i) bulk[i] = 3.0 * lam[i] + 2.0 * mu[i];
  const double* chk[3] = {rho_inv, mu, bulk.data()};
  const char* names[3] = {"1/rho", "mu", "3 lambda + 2 mu"};
  for (int f = 0; f < 3; ++f) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(src[f][i])) return fail(BBWADG_EC2, "medium %d coefficient %zu not finite", f, i);
    PositivityCount pc;
    if ((rc = classify_positive(chk[f], c->M, c->K, pc, names[f]))) return rc;
    if (c->c2_policy == BBWADG_C2_REQUIRE_POSITIVE && pc.nonpositive + pc.undecided > 0)
      return fail(BBWADG_EC2, "%s is not positive everywhere on %lld elements (first element %lld)", names[f],
                  (long long)(pc.nonpositive + pc.undecided), (long long)pc.first);
  }
  // upload into fresh buffers, then replace the old ones: a failure leaves the old media
  void* fresh[3] = {nullptr, nullptr, nullptr};
  for (int f = 0; f < 3 && !rc; ++f) {
    rc = dmalloc(&fresh[f], n * c->rsz);
    if (rc) break;
    if (c->dtype == BBWADG_F64) {
      rc = upload(fresh[f], src[f], n * 8);
    } else {
      std::vector<float> v(src[f], src[f] + n);
      rc = upload(fresh[f], v.data(), n * 4);
    }
  }
  if (rc) {
    for (void* p : fresh)
      if (p) (void)hipFree(p);
    return rc;
  }
  void** dst[3] = {&c->d_el_rho, &c->d_el_lam, &c->d_el_mu};
  for (int f = 0; f < 3; ++f) {
    if (*dst[f]) (void)hipFree(*dst[f]);
    *dst[f] = fresh[f];
  }
  return 0;
}

int bbwadg_elastic_update(bbwadg_ctx* c, const void* r, void* out, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!r || !out) return fail(BBWADG_EINVAL, "NULL state pointer");
  if (r == out) return fail(BBWADG_EINVAL, "r and out must not overlap");
  if (!c->d_el_rho) return fail(BBWADG_EC2, "elastic media not set (call bbwadg_elastic_set_media)");
  return elastic_update_launch(c, r, out, nullptr, nullptr, 0.0, 0.0, 0.0, stream);
}

int bbwadg_adjoint_apply(bbwadg_ctx* c, const void* z, void* out, void* stream) {
  int rc = require_device(c);
  if (rc) return rc;
  if (!z || !out) return fail(BBWADG_EINVAL, "NULL state pointer");
  if (z == out) return fail(BBWADG_EINVAL, "z and out must not overlap");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = sync_c2(c, s)) || (rc = adjoint_setup(c))) return rc;
  const size_t n1 = (size_t)c->K * c->Np, n4 = 4 * n1, rb = c->rsz;
  Scratch ws;
  void* w4;
  if ((rc = ws.get(&w4, n4 * rb))) return rc;
  // w4 = (W z_p, z_u)
  rc = c->dtype == BBWADG_F64 ? wadg_apply<double>(c, z, w4, s) : wadg_apply<float>(c, z, w4, s);
  if (rc ||
      (rc = hip_check(hipMemcpyAsync((char*)w4 + n1 * rb, (const char*)z + n1 * rb, 3 * n1 * rb, hipMemcpyDeviceToDevice, s),
                      "copy u")))
    return rc;
  rc = c->dtype == BBWADG_F64
           ? stage_custom<double>(c, 0, c->d_adj_ones, nullptr, 0.0, false, w4, out, nullptr, 0, 0, 0, s)
           : stage_custom<float>(c, 0, c->d_adj_ones, nullptr, 0.0, false, w4, out, nullptr, 0, 0, 0, s);
  if (rc) return rc;
  return hip_check(hipStreamSynchronize(s), "sync");  // the temporaries are freed on return
}

}  // extern "C"
