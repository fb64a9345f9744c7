/*
 * bbwadg.h -- C ABI of the MI355X (gfx950) BBWADG library.
 *
 * Bernstein-Bezier weight-adjusted DG (BBWADG) for the 3D acoustic system
 *     (1/c^2) p_t + div u = 0,   u_t + grad p = 0          (paper Section 3.1, eq. awave)
 * on affine tetrahedra: right-hand side and low-storage RK4 step.
 *
 * Data format
 * -----------
 * State arrays hold Bernstein coefficients, field-major: q[4][K][Np] with fields
 * (p, u, v, w), Np = (N+1)(N+2)(N+3)/6, element k contiguous within a field, in the
 * context's dtype (double for BBWADG_F64, float for BBWADG_F32).
 * Coefficient i of element k is the coefficient of B^N_alpha (paper Section 2,
 * B^N_alpha = N!/alpha! lambda^alpha) where the barycentric coordinates lambda_0..3
 * belong to the element's vertices SORTED BY ASCENDING GLOBAL VERTEX ID
 * (bbwadg_element_vertices returns that order), and alpha = (a0,a1,a2,a3) is
 * enumerated graded by s = a1+a2+a3 (0..N), then a3 ascending, then a2 ascending
 * (a1 = s-a2-a3, a0 = N-s); the index of (a1,a2,a3) is then
 *     dimp(s-1) + a3 (2s+3-a3)/2 + a2,   dimp(n) = (n+1)(n+2)(n+3)/6, dimp(-1) = 0,
 * independent of N. The same order is used for c^2 coefficients of degree M:
 * c2[K][Mp], Mp = (M+1)(M+2)(M+3)/6.
 *
 * Ownership and streams
 * ---------------------
 * The caller owns every state/rhs/res/c2 buffer passed in; the library never frees
 * them. The library owns the context: geometry, connectivity, operator tables, the
 * per-element c^2 coefficients and one internal state-sized device buffer, all
 * allocated by bbwadg_create and freed by bbwadg_destroy. bbwadg_rhs and bbwadg_step
 * allocate nothing. Streams are borrowed hipStream_t values passed as void*
 * (NULL = the null stream); all device work is asynchronous on that stream.
 * A context is not thread-safe: the caller serialises calls on one context.
 *
 * Errors
 * ------
 * Every entry point returns 0 (BBWADG_OK) or a negative code; bbwadg_last_error()
 * returns a thread-local message for the last failure. On error no state changes.
 */
#ifndef BBWADG_H
#define BBWADG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BBWADG_OK = 0,
  BBWADG_EINVAL = -1, /* bad argument: range, NULL pointer, dtype, host-only context */
  BBWADG_EMESH = -2,  /* non-conforming mesh, face shared by > 2 elements, degenerate element */
  BBWADG_EC2 = -3,    /* c^2 (or an elastic medium) not set, non-finite, or not positive
                         everywhere on an element (see bbwadg_set_c2_policy) */
  BBWADG_ENOMEM = -4, /* host or device allocation failed */
  BBWADG_EHIP = -5    /* HIP runtime or kernel launch error */
};

enum { BBWADG_F64 = 0, BBWADG_F32 = 1 };
enum { BBWADG_BC_P0 = 0, BBWADG_BC_RIGID = 1 };
enum { BBWADG_DEVICE = 0, BBWADG_HOST_ONLY = 1 };
enum { BBWADG_C2_REQUIRE_POSITIVE = 0, BBWADG_C2_ACCEPT_NONPOSITIVE = 1 };

typedef struct bbwadg_ctx bbwadg_ctx;

typedef struct {
  int64_t num_vertices;  /* Nv */
  const double* xyz;     /* host [Nv][3], copied */
  int64_t num_elements;  /* K >= 1 */
  const int32_t* etov;   /* host [K][4] vertex ids in [0, Nv), any order; copied */
  int32_t bc;            /* boundary faces: BBWADG_BC_P0 (p+ = -p, u+ = u) or
                            BBWADG_BC_RIGID (p+ = p, u+ = u - 2(u.n)n) */
} bbwadg_mesh;

typedef struct {
  int32_t N;       /* polynomial degree, 1..9 */
  int32_t M;       /* degree of the c^2 approximation, 0..min(N,4) */
  int32_t dtype;   /* BBWADG_F64 or BBWADG_F32: storage and arithmetic of rhs/step */
  int32_t mode;    /* BBWADG_DEVICE, or BBWADG_HOST_ONLY (geometry, tables and projections
                      only; no HIP call is made and rhs/step return BBWADG_EINVAL) */
  double tau_p;    /* penalty on [[p]] (paper Section 3.1 fluxes), >= 0 */
  double tau_u;    /* penalty on [[u]].n, >= 0 */
} bbwadg_opts;

/* Build a context: sorts each element's vertices by global id, computes the affine
 * geometry (G = dr/dx, J = |det dx/dr|, outward unit normals, Fscale = J_f/J with
 * J_f = face area / 2), matches faces by their vertex triple, builds the Bernstein
 * operator tables and (device mode) uploads them. Paper Section 3.1, eq. (matform).
 * Errors: EINVAL (NULL, N/M/dtype/tau out of range, vertex id out of range),
 * EMESH (face shared by more than two elements, |det| <= 1e-14 * h^3), ENOMEM, EHIP. */
int bbwadg_create(const bbwadg_mesh* mesh, const bbwadg_opts* opts, bbwadg_ctx** out);

/* Free a context and its device buffers (NULL is a no-op). Synchronises the device. */
int bbwadg_destroy(bbwadg_ctx* ctx);

/* Thread-local text of the last error ("" if none). Valid until the next call. */
const char* bbwadg_last_error(void);

/* Sizes: Np, Nfp = (N+1)(N+2)/2, Mp, K. Any pointer may be NULL. */
int bbwadg_sizes(const bbwadg_ctx* ctx, int32_t* Np, int32_t* Nfp, int32_t* Mp, int64_t* K);

/* The element-to-vertex list in the library's local order (ascending global id per
 * element), host [K][4]. This order defines the barycentric coordinates. */
int bbwadg_element_vertices(const bbwadg_ctx* ctx, int32_t* etov_out);

/* Per-element geometry, host arrays (any may be NULL): J [K]; G [K][3][3] with
 * G[k][i][j] = d r_j / d x_i; normal [K][4][3] outward unit normal of face f (face f is
 * opposite local vertex f); Fscale [K][4] = J_f / J; nbr [K][4] = 4*k'+f' of the
 * neighbour element k' and its face f', or -1 on the boundary. */
int bbwadg_geometry(const bbwadg_ctx* ctx, double* J, double* G, double* normal, double* Fscale,
                    int32_t* nbr);

/* ---- L^2 projections onto Bernstein polynomials (setup; FP64 on the host) ----
 * A function f is projected per element onto P^d by the collapsed Gauss-Jacobi rule
 * with n = d+3 points per direction (exact to degree 2d+5): coef = M_d^{-1} B^T W f.
 * The caller samples f at the physical points and passes the samples back, so any
 * Python/C function can be used. Elements are processed in ranges [k0, k1).        */

/* Number of projection points per element for target degree d = M (c^2) or N (state). */
int bbwadg_projection_npoints(const bbwadg_ctx* ctx, int32_t degree, int64_t* nq);

/* Physical projection points of elements [k0,k1) for degree d: host [k1-k0][nq][3]. */
int bbwadg_projection_points(const bbwadg_ctx* ctx, int32_t degree, int64_t k0, int64_t k1,
                             double* xyz_out);

/* Project samples host [k1-k0][nq] onto degree d; writes host FP64 [k1-k0][dimp(d)]. */
int bbwadg_project_samples(const bbwadg_ctx* ctx, int32_t degree, int64_t k0, int64_t k1,
                           const double* samples, double* coef_out);

/* c^2 setup (paper Section 5: c^2 replaced by its per-element L^2 projection onto P^M).
 * bbwadg_project_c2 samples the callback c2(x, y, z, user) at the projection points,
 * projects in FP64, checks the result like bbwadg_set_c2, stores the coefficients in the
 * context and, if c2_out != NULL, copies them as dtype into the device buffer c2_out
 * [K][Mp] on `stream`. Stream-ordered before later rhs/step calls. */
int bbwadg_project_c2(bbwadg_ctx* ctx, double (*c2)(double x, double y, double z, void* user),
                      void* user, void* c2_out, void* stream);

/* Inject per-element c^2 Bernstein coefficients host FP64 [K][Mp] (e.g. shared data for
 * parity runs). The device copy is refreshed on the next rhs/step call.
 * Check (Section 3: the weight-adjusted scheme is energy stable for a positive weight;
 * Section 2: Bernstein polynomials are a nonnegative partition of unity): an element's
 * c^2_M is accepted as positive when all its coefficients are > 0 (the polynomial lies in
 * their convex hull); otherwise its tetrahedron is bisected along the longest edge, with
 * the coefficients of the halves from de Casteljau subdivision, until every piece has
 * positive coefficients (positive), a piece has a vertex value <= 0 (not positive), or
 * 4096 pieces were visited (undecided). Under BBWADG_C2_REQUIRE_POSITIVE (the default)
 * any element not positive or undecided gives EC2 and nothing is stored. EC2 as well for a
 * non-finite value. */
int bbwadg_set_c2(bbwadg_ctx* ctx, const double* c2_coef);

/* Policy of bbwadg_set_c2 / bbwadg_project_c2 / bbwadg_elastic_set_media for a weight that
 * is not positive everywhere: BBWADG_C2_REQUIRE_POSITIVE (default, EC2) or
 * BBWADG_C2_ACCEPT_NONPOSITIVE (stored anyway; the energy bound of the scheme is then lost
 * and the counts below say on how many elements). EINVAL for another value. */
int bbwadg_set_c2_policy(bbwadg_ctx* ctx, int32_t policy);

/* Counts for the stored c^2_M: elements with a value <= 0 and elements left undecided (see
 * bbwadg_set_c2). EC2 if none is set. Either pointer may be NULL. */
int bbwadg_c2_positivity(const bbwadg_ctx* ctx, int64_t* n_nonpositive, int64_t* n_undecided);

/* The same classification for n arbitrary sets of degree-`degree` Bernstein coefficients
 * host FP64 [n][dimp(degree)] (graded order), no context needed: counts of sets not
 * positive / undecided, and the first such set (-1 if none). EINVAL for a bad degree (0..13)
 * or n < 0, EC2 for a non-finite value. Any output pointer may be NULL. */
int bbwadg_bernstein_positivity(int32_t degree, int64_t n, const double* coef, int64_t* n_nonpositive,
                                int64_t* n_undecided, int64_t* first);

/* Read back the stored c^2 coefficients, host FP64 [K][Mp]. EC2 if none is set. */
int bbwadg_get_c2(const bbwadg_ctx* ctx, double* c2_coef);

/* ---- hot path (device) ---- */

/* Right-hand side (paper eq. WADGform, three parts: volume, surface/lift, WADG update):
 *   rhs_p   = Pi_N( c^2_M * ( -div u + sum_f Fscale_f L^f F_p ) )
 *   rhs_u_i = -d p/d x_i + sum_f Fscale_f n_i L^f F_u
 * with F_p = (tau_p [[p]] - n.[[u]])/2 and F_u = (tau_u [[u]].n - [[p]])/2 (paper
 * Section 3.1), derivatives by the sparse Bernstein stencils (Section 4), the lift by
 * L^f = E_L L_0 (Section 4), the c^2 product by eq. (mcoeff) and Pi_N by the telescoped
 * projection eq. (telescope) (Section 5). q, rhs: device [4][K][Np] of dtype, must not
 * overlap. With a pressure source (bbwadg_set_source) r_p gains Pi_N f(., t). */
int bbwadg_rhs(bbwadg_ctx* ctx, const void* q, void* rhs, double t, void* stream);

/* Advance q in place by nsteps steps of the five-stage, 2N-storage fourth-order
 * Runge-Kutta scheme of Carpenter and Kennedy (paper Section 6.3.1): per stage
 * res = a_k res + dt rhs(q), q = q + b_k res. res: device [4][K][Np], the 2N-storage
 * register; zero it before the first step of a run. nsteps >= 0. q and res must not
 * overlap. Stage k of step n is taken at time t0 + (n + c_k) dt (for the source). Each stage is one fused kernel that reads the state from one buffer and
 * writes the next state to the other (q or the context's internal buffer); an odd
 * total stage count ends with one device copy back into q. */
int bbwadg_step(bbwadg_ctx* ctx, void* q, void* res, double t0, double dt, int32_t nsteps,
                void* stream);

/* Pressure source for manufactured solutions (paper Section 6.1): the first equation becomes
 * (1/c^2) p_t + div u = f with f(x, t) = amp sin(omega t + phase) g(x), and the WADG update
 * applies to r_p + Pi_N f, i.e. dp/dt = Pi_N(c^2_M (r_p + Pi_N f)). g: host FP64 Bernstein
 * coefficients [K][Np] of Pi_N g (e.g. from bbwadg_project_samples with degree N), copied;
 * NULL removes the source. EINVAL for non-finite input. */
int bbwadg_set_source(bbwadg_ctx* ctx, const double* g, double amp, double omega, double phase);

/* dt = cfl / (c_max C_N max_{k,f} Fscale), C_N = (N+1)(N+3)/3, c_max^2 = the largest
 * c^2 Bernstein coefficient (an upper bound of c^2_M by the convex-hull property). */
int bbwadg_suggest_dt(const bbwadg_ctx* ctx, double cfl, double* dt);

/* Per-field squared L^2 norms sum_k J_k int_ref q_k^2 of a device state [4][K][Np],
 * accumulated in FP64 on the device with the closed-form Bernstein mass matrix;
 * out: host double[4]. Synchronises `stream`. */
int bbwadg_l2norm2(bbwadg_ctx* ctx, const void* q, double out[4], void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): bbwadg_l2norm2 with no allocation and no
 * synchronisation. The per-block partial sums go to a fixed device array of the library
 * (1,024 blocks x 4 doubles = 32 KiB on each GPU the library runs on, held until the
 * process ends) and a second kernel adds them in block order into out, so the result equals
 * bbwadg_l2norm2's bit for bit. q: device [4][K][Np] of the context dtype; out: device
 * double[4], written asynchronously on `stream`. Every call on one GPU shares that array
 * (each call writes all of the partial sums it reads), so calls that overlap on one GPU,
 * e.g. on two streams, race. EINVAL for NULL arguments or when the current device is not
 * the context's; EHIP for a launch error. */
int bbwadg_l2norm2_noalloc(bbwadg_ctx* ctx, const void* q, double* out, void* stream);

/* ---- FP64 quadrature reductions (L^2 errors as in the convergence study of paper
 * Section 6.1; the acoustic energy of eq. (awave), in which WADG is stable, Section 3) ----
 * Both evaluate the device state q [4][K][Np] at the points of the degree-N projection rule
 * (the points bbwadg_projection_points(ctx, N, ...) returns, in that order; nq = (N+3)^3
 * per element; exact for polynomials of degree 2N+5) and accumulate in FP64 whatever the
 * context's dtype. They cover elements [k0, k1), so a large mesh can be reduced in pieces
 * whose results add; k0 == k1 gives zeros. The host sums per-block partials in a fixed
 * order (deterministic). Synchronise `stream`. EINVAL on a bad range or NULL pointer. */

/* out[f] = sum_{k0<=k<k1} J_k sum_q w_q (q_f(x_q) - exact[f][k-k0][q])^2, the squared L^2
 * error of field f against a reference solution that the caller sampled at the rule points.
 * exact: device FP64 [4][k1-k0][nq], caller-owned. */
int bbwadg_l2error2(bbwadg_ctx* ctx, const void* q, int64_t k0, int64_t k1, const double* exact,
                    double out[4], void* stream);

/* Acoustic energy (1/2) int (p^2 / c^2_M + |u|^2) over elements [k0, k1), returned per term:
 * out[0] = the p^2/c^2_M term, out[1..3] = the u, v, w terms (the energy is their sum), with
 * the context's stored c^2_M (EC2 if none). Where c^2_M is constant on an element this equals
 * the weight-adjusted energy (1/2)(p^T M M_{c^2}^{-1} M p + u^T M u) of the semi-discrete
 * scheme; otherwise it bounds that quantity from above (Cauchy-Schwarz). */
int bbwadg_energy(bbwadg_ctx* ctx, const void* q, int64_t k0, int64_t k1, double out[4], void* stream);

/* Project fn(x, y, z, user) onto P^N per element (the degree-N projection rule, FP64 on the
 * host, as in bbwadg_project_samples) and write the coefficients, converted to dtype, as field
 * `field` (0 = p, 1..3 = u, v, w) of the device state q_out [4][K][Np]; the other fields are
 * untouched. Initial conditions, paper Section 6. EINVAL for a non-finite sample or a field
 * outside 0..3. Synchronises `stream`. */
int bbwadg_project_fn(bbwadg_ctx* ctx, double (*fn)(double x, double y, double z, void* user),
                      void* user, int32_t field, void* q_out, void* stream);

/* ---- dense quadrature WADG: the comparison baseline (paper Section 3.3, eq. pwadg) ----
 * dp/dt = P_q diag(c^2(x_q)) V_q r_p with V_q the degree-N Bernstein basis at the points of
 * the collapsed Gauss-Jacobi rule with n = floor((2N+M+2)/2) points per direction (exact to
 * degree 2N+M) and P_q = M^{-1} V_q^T W, applied as dense products on the matrix cores in
 * the context's precision (FP64, or FP32 with FP32 accumulation). With c^2_M at the points it
 * equals the fast Bernstein update (paper Theorem 5.3); with the true c^2 at the points it is
 * the quadrature WADG the paper compares against. Device contexts only. The point values take
 * K * 16 ceil(nq/16) reals of device memory, allocated by the first bbwadg_dense_set_c2
 * together with the tables. */

/* Points of the dense rule per element (nq = n^3). */
int bbwadg_dense_npoints(const bbwadg_ctx* ctx, int64_t* nq);

/* Physical points of the dense rule for elements [k0, k1): host [k1-k0][nq][3]. */
int bbwadg_dense_points(const bbwadg_ctx* ctx, int64_t k0, int64_t k1, double* xyz_out);

/* Set c^2 at the dense points: host FP64 [K][nq] (in bbwadg_dense_points' order), or NULL to
 * evaluate the stored c^2_M there. EC2 if a value is not finite and positive, or if c2q is
 * NULL and no c^2_M is set. Synchronises `stream`. */
int bbwadg_dense_set_c2(bbwadg_ctx* ctx, const double* c2q, void* stream);

/* The dense update alone: out[k] = P_q diag(c^2 at element k's points) V_q r[k] for device
 * arrays r, out [K][Np] of the context dtype (they may be the same array). EC2 before
 * bbwadg_dense_set_c2. */
int bbwadg_dense_update(bbwadg_ctx* ctx, const void* r, void* out, void* stream);

/* Right-hand side with the dense update in place of the Bernstein one: the plain DG
 * right-hand side (volume, fluxes and lift as in bbwadg_rhs, with c^2 = 1) followed by
 * bbwadg_dense_update on the p field. q, rhs: device [4][K][Np] of the context dtype, must
 * not overlap. */
int bbwadg_rhs_dense(bbwadg_ctx* ctx, const void* q, void* rhs, double t, void* stream);

/* ---- receivers, misfit and its gradient with respect to c^2_M -------------------------
 * Receivers sample the pressure after each step; the misfit of a run of nsteps steps is
 * J = 1/2 sum_n sum_r (p(x_r, t_n) - d[n][r])^2. Its gradient with respect to the
 * per-element Bernstein coefficients of c^2_M (the weight of the weight-adjusted projection,
 * paper Section 3.1 and Section 5) is the exact discrete adjoint of the LSRK4 scheme. */

/* Place nrec receivers at host FP64 points xyz [nrec][3]. Each lies in the lowest-numbered
 * element whose barycentric coordinates are all >= -1e-10 (the pressure is discontinuous
 * across elements, so a point on a shared face takes that element's value). The library keeps
 * copies of the basis values there and of the row of (J_k M)^{-1}, M the Bernstein mass matrix.
 * nrec = 0 removes them. EINVAL for a point outside the mesh or a non-finite coordinate. Works
 * on host-only contexts (no device copies). */
int bbwadg_set_receivers(bbwadg_ctx* ctx, int32_t nrec, const double* xyz);

/* Host int32[nrec]: the element of each receiver. */
int bbwadg_receiver_elements(const bbwadg_ctx* ctx, int32_t* elem_out);

/* Run nsteps LSRK4 steps from the device state q0 [4][K][Np] (not modified; the source, if
 * set, enters at the stage times t0 + (n + c_k) dt) and return the misfit in *misfit (host).
 * data: device FP64 [nsteps][nrec] observed traces, or NULL for zeros. traces: device FP64
 * [nsteps][nrec] for the computed traces, or NULL. grad: device FP64 [K][Mp] for dJ/dc (overwritten), or NULL
 * to stop after the forward run.
 *
 * The backward pass takes the transposed stages in reverse order in the variables
 * z = (M S)^{-1} lambda (S = diag(1, -1, -1, -1) reflects the velocity, M is the block mass
 * matrix): the DG operator's symmetric part is the penalty alone, which does not couple p and
 * u, so A^T (M S) = (M S) B W with B the plain DG operator and W the weight-adjusted
 * projection, and each transposed stage is one update launch (W, as bbwadg_wadg_update) and
 * one stage-kernel launch (B). The forward states are
 * checkpointed every checkpoint_every steps and each segment is recomputed once; its update
 * launches also store the pressure part of B q (r_p before the weight adjustment) of its
 * 5 checkpoint_every stages. Device memory allocated and freed
 * inside the call: about (3 + nsteps/checkpoint_every) states and, with grad, the pressure
 * part of 5 checkpoint_every stages and 4 states more; synchronises `stream`. EINVAL without receivers. */
int bbwadg_misfit_gradient(bbwadg_ctx* ctx, const void* q0, double t0, double dt, int32_t nsteps, const double* data,
                           int32_t checkpoint_every, double* traces, double* misfit, double* grad, void* stream);

/* The transposed operator in the variables of bbwadg_misfit_gradient: out = B(W z), i.e.
 * A^T (M S z) = M S out. For device states z, out [4][K][Np] of the context dtype (no
 * overlap). Allocates one state-sized temporary; synchronises `stream`. */
int bbwadg_adjoint_apply(bbwadg_ctx* ctx, const void* z, void* out, void* stream);

/* The weight-adjusted update on its own (paper Section 5, the update kernel of Table am1):
 * out = Pi_N(c^2_M r), the product with c^2_M exact in degree N + M (eq. mcoeff) and Pi_N the
 * telescoped projection (Theorem 5.3). r, out: device [K][Np] of the context dtype, no
 * overlap. EC2 without c^2. The fused stage kernel computes the same update internally. */
int bbwadg_wadg_update(bbwadg_ctx* ctx, const void* r, void* out, void* stream);

/* ---- elastic weight-adjusted update (paper Section 3.2, eq. ewadg) ----------------------
 * The velocity-stress system rho v_t = sum_i A_i^T d sigma/dx_i, C^{-1} sigma_t = sum_i A_i
 * dv/dx_i with isotropic C (Lame parameters lambda, mu). Its weighted mass matrices are
 * replaced by the weight-adjusted inverse (I (x) M^{-1}) M_C (I (x) M^{-1}) (and M_{1/rho}
 * for the velocity), applied with the context's N, M and telescoped projection. */

/* Media: host FP64 Bernstein coefficients [K][Mp] of degree M of 1/rho, lambda and mu (e.g.
 * projections from bbwadg_project_samples with degree M), copied. The mass-matrix weights
 * 1/rho, mu and 3 lambda + 2 mu must be positive everywhere (the check of bbwadg_set_c2,
 * under the same policy); all three are checked before any is uploaded, and on an error
 * the previous media stay in place. EC2 for a non-finite or not positive medium. */
int bbwadg_elastic_set_media(bbwadg_ctx* ctx, const double* rho_inv, const double* lam, const double* mu);

/* out = the weight-adjusted update of the DG right-hand side r, both device [9][K][Np] of the
 * context dtype (v1, v2, v3, sigma_xx, yy, zz, yz, xz, xy), no overlap:
 *   out_v_i = Pi_N(rho^{-1} r_v_i),  out_sigma_i = Pi_N(lambda tr r_sigma + 2 mu r_sigma_i)
 *   (i = xx, yy, zz),  out_sigma_s = Pi_N(mu r_sigma_s)  (s = yz, xz, xy),
 * each product exact in degree N + M (eq. mcoeff) and each Pi_N the telescoped projection
 * (Theorem 5.3): 12 products and 9 scalar projections per element. EC2 before
 * bbwadg_elastic_set_media. */
int bbwadg_elastic_update(bbwadg_ctx* ctx, const void* r, void* out, void* stream);

/* The elastic DG right-hand side (paper Section 3.2, the semi-discrete form after eq. ewave)
 * with upwind-type penalty fluxes, A_n = sum_i n_i A_i on each face:
 *   r_v = sum_i A_i^T d sigma/dx_i + sum_f (J_f/J) L^f F_v,  F_v = A_n^T [[sigma]]/2 + tau_v/2 A_n^T A_n [[v]]
 *   r_s = sum_i A_i   d v/dx_i     + sum_f (J_f/J) L^f F_s,  F_s = A_n [[v]]/2     + tau_s/2 A_n A_n^T [[sigma]]
 * ([[u]] = u+ - u-, L^f the lift of face f). Boundary faces take the mirror state of `wall`:
 * 0 traction-free (sigma+ = -sigma, v+ = v), 1 rigid (v+ = -v, sigma+ = sigma). q, rhs: device
 * [9][K][Np] of the context dtype, no overlap. weighted = 0 returns the right-hand side before
 * the media enter; weighted = 1 follows it with bbwadg_elastic_update (EC2 before
 * bbwadg_elastic_set_media) through a context-owned [9][K][Np] temporary, allocated on the first
 * such call. EINVAL for a bad wall or a negative or non-finite tau. The lift is the factored
 * Bernstein lift of Section 4 (L_0 and a chain of 2D degree reductions); a face-position table
 * is uploaded on the first call. */
int bbwadg_elastic_rhs(bbwadg_ctx* ctx, const void* q, void* rhs, int32_t wall, double tau_v, double tau_s,
                       int32_t weighted, void* stream);

/* nsteps low-storage RK4 steps (the 5-stage 2N-storage scheme of Carpenter and Kennedy that the
 * acoustic step uses) of the elastic system: per stage res = a_k res + dt r(q), q += b_k res with
 * r the weighted right-hand side of bbwadg_elastic_rhs (wall, tau_v, tau_s as there). q, res:
 * device [9][K][Np] of the context dtype, updated in place, no overlap; res starts at zero for a
 * fresh run. EC2 before bbwadg_elastic_set_media; EINVAL for dt <= 0, nsteps < 0. */
int bbwadg_elastic_step(bbwadg_ctx* ctx, void* q, void* res, double dt, int32_t nsteps, int32_t wall, double tau_v,
                        double tau_s, void* stream);

/* Position of the Bernstein coefficient with multi-index (n - a1 - a2 - a3, a1, a2, a3) in the
 * coefficient order documented above; it does not depend on the degree n >= a1 + a2 + a3
 * (paper Section 2 defines the multi-indices). EINVAL for a negative entry or a1+a2+a3 > 13. */
int32_t bbwadg_coef_index(int32_t a1, int32_t a2, int32_t a3);

/* c_j of the telescoped projection P^{N+M}_N = sum_j c_j E^N_{N-j}(E^N_{N-j})^T
 * (E^{N+M}_N)^T (paper Theorem 5.3, Table 1), host double[N+1]. With M < 0 returns the
 * coefficients of the inverse mass matrix representation (paper Theorem 5.5, Table 2).
 * 1 <= N <= 9, -1 <= M <= 9. */
int bbwadg_projection_coefficients(int32_t N, int32_t M, double* cj_out);

/* Library version string. */
const char* bbwadg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BBWADG_H */
