"""Quadrature-based weight-adjusted DG for the 3D acoustic system (the oracle proper).

Test infrastructure only (see the package docstring).

Semi-discrete form (paper Section 3.1, eq. (sdf) and (WADGform); the sign of the lift term
in (WADGform) is read as in (matform): only the volume term is negated):

    r_p   = -div u  + sum_f (J_f/J) L^f F_p,     F_p = (tau_p [[p]] - n.[[u]]) / 2
    r_u_i = -d_i p  + sum_f (J_f/J) n_i L^f F_u,  F_u = (tau_u [[u]].n - [[p]]) / 2
    dp/dt = M^{-1} M_{c^2} r_p = P_q diag(c^2(x_q)) V_q r_p          (eq. pwadg)
    du_i/dt = r_u_i

with D_j = M^{-1} S_j, L^f = M^{-1} M_f and P_q = M^{-1} V_q^T W, all formed by
quadrature in an orthonormal basis. [[q]] = q+ - q. Boundary faces use mirror states:
p = 0 walls take p+ = -p, u+ = u; rigid walls take p+ = p, u+ = u - 2 (u.n) n.

The weight c^2 is read as c^2 (not 1/c^2): the weight-adjusted inverse of M_{1/c^2} is
M^{-1} M_{c^2} M^{-1} (paper Section 3.1), and the experiments project c^2 (Section 6.1).
"""
from __future__ import annotations

import numpy as np

from .basis import bernstein_tet, dubiner_tet
from .mesh import Mesh
from .quadrature import points_for_degree, tet_rule, tri_rule

# Carpenter & Kennedy (1994), five-stage 2N-storage fourth-order scheme, the
# low-storage RK4 named in paper Section 6.3.1.
LSRK4_A = (0.0,
           -567301805773.0 / 1357537059087.0,
           -2404267990393.0 / 2016746695238.0,
           -3550918686646.0 / 2091501179385.0,
           -1275806237668.0 / 842570457699.0)
LSRK4_B = (1432997174477.0 / 9575080441755.0,
           5161836677717.0 / 13612068292357.0,
           1720146321549.0 / 2090206949498.0,
           3134564353537.0 / 4481467310338.0,
           2277821191437.0 / 14882151754819.0)
LSRK4_C = (0.0,
           1432997174477.0 / 9575080441755.0,
           2526269341429.0 / 6820363183787.0,
           2006345519317.0 / 3224310063776.0,
           2802321613138.0 / 2924317926251.0)


def _tet_points_from_lambda(lam):
    """(r, s, t) of barycentric coordinates lam [4, npts]."""
    return 2.0 * lam[1] - 1.0, 2.0 * lam[2] - 1.0, 2.0 * lam[3] - 1.0


def dim_p(n):
    return (n + 1) * (n + 2) * (n + 3) // 6


class Oracle:
    """Dense quadrature WADG on a given mesh, degree N, c^2 weight of degree M."""

    def __init__(self, xyz, etov, N: int, M: int, tau_p: float = 1.0, tau_u: float = 1.0,
                 bc: str = "p0", mesh: Mesh | None = None):
        if bc not in ("p0", "rigid"):
            raise ValueError("bc must be 'p0' or 'rigid'")
        self.mesh = mesh if mesh is not None else Mesh(xyz, etov)
        self.N, self.M = int(N), int(M)
        self.Np = dim_p(N)
        self.tau_p, self.tau_u, self.bc = float(tau_p), float(tau_u), bc
        N = self.N
        # volume rule exact to degree 2N+M (mass with weight c^2_M), face rule exact to 2N
        nq = points_for_degree(2 * N + self.M)
        r, s, t, w = tet_rule(nq)
        self.rq, self.sq, self.tq, self.wq = r, s, t, w
        V, (Vr, Vs, Vt) = dubiner_tet(N, r, s, t, grad=True)
        self.Vq = V
        Mref = V.T @ (w[:, None] * V)
        self.Mref = Mref
        self.Minv = np.linalg.inv(Mref)
        self.Pq = self.Minv @ (V.T * w[None, :])
        self.D = [self.Minv @ (V.T @ (w[:, None] * Vd)) for Vd in (Vr, Vs, Vt)]
        # faces
        r2, s2, wf = tri_rule(N + 1)
        self.wf = wf
        mu = np.stack([-(r2 + s2) / 2.0, (1.0 + r2) / 2.0, (1.0 + s2) / 2.0])
        self.mu = mu
        self.Vf, self.Lf = [], []
        for f in range(4):
            lam = np.zeros((4, mu.shape[1]))
            for m, v in enumerate(self.mesh.face_local[f]):
                lam[v] = mu[m]
            Vf = dubiner_tet(N, *_tet_points_from_lambda(lam))
            self.Vf.append(Vf)
            self.Lf.append(self.Minv @ (Vf.T * wf[None, :]))
        self._build_neighbour_groups()
        self.c2q = None
        self.src = None

    # ------------------------------------------------------------- neighbours
    def _build_neighbour_groups(self):
        """Group interior faces by where the neighbour holds the shared vertices.

        A face point with barycentrics mu on this element's face vertices has the same
        barycentrics on the same global vertices of the neighbour, so the neighbour's
        polynomial is evaluated at reference points built from those positions.
        """
        msh = self.mesh
        self.groups = []
        self.bmask = []
        for f in range(4):
            interior = msh.nbr[:, f] >= 0
            self.bmask.append(~interior)
            keys = {}
            ks = np.nonzero(interior)[0]
            pos = msh.nbr_pos[ks, f]
            for key in set(map(tuple, pos.tolist())):
                sel = ks[np.all(pos == np.array(key)[None, :], axis=1)]
                lam = np.zeros((4, self.mu.shape[1]))
                for m in range(3):
                    lam[key[m]] = self.mu[m]
                Vn = dubiner_tet(self.N, *_tet_points_from_lambda(lam))
                keys[key] = (sel, msh.nbr[sel, f], Vn)
            self.groups.append(list(keys.values()))

    # ----------------------------------------------------------------- c^2 setup
    def set_c2_bernstein(self, coef):
        """c^2_M given as per-element Bernstein coefficients [K, M_p] of degree M."""
        coef = np.asarray(coef, dtype=np.float64).copy()
        self._c2_ref = lambda r, s, t: coef @ bernstein_tet(self.M, r, s, t).T
        self.c2q = self._c2_ref(self.rq, self.sq, self.tq)

    def set_c2_function(self, fn, project: bool = True, nproj: int | None = None):
        """c^2 from a function: its per-element L^2 projection onto P^M (the fast method's
        input, paper Section 5) or, with ``project=False``, its point values (plain WADG)."""
        if not project:
            def at(r, s, t):
                X = self.mesh.map_points(r, s, t)
                return np.broadcast_to(fn(X[..., 0], X[..., 1], X[..., 2]), X.shape[:-1])
        else:
            modal = self.project_modal(fn, self.M, nproj)
            def at(r, s, t):
                return modal @ dubiner_tet(self.M, r, s, t).T
        self._c2_ref = at
        self.c2q = at(self.rq, self.sq, self.tq)

    def c2_at(self, r, s, t):
        """c^2 as set, at reference points (r, s, t) of every element: [K, npts]."""
        if self.c2q is None:
            raise RuntimeError("c^2 not set")
        return self._c2_ref(np.atleast_1d(r), np.atleast_1d(s), np.atleast_1d(t))

    def project_modal(self, fn, deg: int, nproj: int | None = None):
        """Per-element L^2 projection of fn onto P^deg, as orthonormal-basis coefficients.

        Uses the collapsed Gauss-Jacobi rule with deg + 3 points per direction (exact to
        degree 2 deg + 5) unless ``nproj`` is given. The paper does not fix the rule for
        this projection; this one is the reading shared with the library's setup code.
        """
        n = deg + 3 if nproj is None else nproj
        r, s, t, w = tet_rule(n)
        V = dubiner_tet(deg, r, s, t)
        Mm = V.T @ (w[:, None] * V)
        P = np.linalg.solve(Mm, V.T * w[None, :])
        X = self.mesh.map_points(r, s, t)
        vals = fn(X[..., 0], X[..., 1], X[..., 2])  # [K, nq]
        return vals @ P.T

    def project_to_quad(self, fn, deg, nproj=None):
        coef = self.project_modal(fn, deg, nproj)
        Vd = dubiner_tet(deg, self.rq, self.sq, self.tq)
        return coef @ Vd.T

    # ------------------------------------------------------------- conversions
    def from_bernstein(self, bern):
        """Orthonormal-basis coefficients of Bernstein coefficient arrays [..., K, Np]."""
        B = bernstein_tet(self.N, self.rq, self.sq, self.tq)
        T = self.Pq @ B  # exact: quadrature integrates degree 2N exactly
        return np.asarray(bern, dtype=np.float64) @ T.T

    def project_initial(self, fns):
        """State [4, K, Np] from four functions (p, u, v, w) of (x, y, z)."""
        return np.stack([self.project_modal(f, self.N) for f in fns])

    def values_at_quad(self, Q):
        return Q @ self.Vq.T

    def bernstein_values_at_quad(self, bern):
        B = bernstein_tet(self.N, self.rq, self.sq, self.tq)
        return np.asarray(bern, dtype=np.float64) @ B.T

    def l2_sq(self, vals):
        """Per-field squared L^2 norms over the mesh of values at the volume points."""
        wJ = self.mesh.J[:, None] * self.wq[None, :]
        return np.sum(vals * vals * wJ, axis=(-1, -2))

    def rel_l2(self, vals_a, vals_b):
        """Per-field ||a - b|| / ||b|| over the mesh."""
        return np.sqrt(self.l2_sq(vals_a - vals_b) / np.maximum(self.l2_sq(vals_b), 1e-300))

    # ---------------------------------------------------------------------- RHS
    def traces(self, Q, f):
        """Own and neighbour traces of all 4 fields at face f's points: two [4, K, Nfq]."""
        own = Q @ self.Vf[f].T
        nb = np.empty_like(own)
        for sel, ks2, Vn in self.groups[f]:
            nb[:, sel] = Q[:, ks2] @ Vn.T
        bm = self.bmask[f]
        if np.any(bm):
            n = self.mesh.normal[bm, f]  # [Kb, 3]
            if self.bc == "p0":
                nb[0, bm] = -own[0, bm]
                nb[1:, bm] = own[1:, bm]
            else:
                un = np.einsum("ikq,ki->kq", own[1:, bm], n)
                nb[0, bm] = own[0, bm]
                nb[1:, bm] = own[1:, bm] - 2.0 * un[None] * n.T[:, :, None]
        return own, nb

    def set_source(self, g_fn, amp: float = 1.0, omega: float = 0.0, phase: float = 0.0, nproj=None):
        """Pressure source f(x, t) = amp sin(omega t + phase) g(x): the first equation becomes
        (1/c^2) p_t + div u = f (the manufactured solutions of paper Section 6.1). Read as
        dp/dt = Pi_N(c^2 (r_p + Pi_N f)) with Pi_N f the per-element L^2 projection. ``g_fn``
        is a vectorised function or the orthonormal coefficients [K, Np] of Pi_N g."""
        if callable(g_fn):
            self.src = self.project_modal(g_fn, self.N, nproj)
        else:
            self.src = np.array(g_fn, dtype=np.float64).reshape(self.mesh.K, self.Np)
        self.src_time = (float(amp), float(omega), float(phase))

    def source_factor(self, t: float) -> float:
        if self.src is None:
            return 0.0
        amp, omega, phase = self.src_time
        return amp * np.sin(omega * t + phase)

    def rhs(self, Q, pre_wadg: bool = False, t: float = 0.0):
        """Time derivative of the state Q [4, K, Np] (orthonormal coefficients) at time t.

        With ``pre_wadg`` the p-component is r_p (with the source, if any), before the
        weight-adjusted step."""
        Q = np.asarray(Q, dtype=np.float64)
        msh = self.mesh
        G = msh.G
        dQ = [Q @ Dj.T for Dj in self.D]  # d/dr_j of all fields, each [4, K, Np]
        rp = np.zeros_like(Q[0])
        ru = np.zeros_like(Q[1:])
        for i in range(3):
            for j in range(3):
                g = G[:, i, j][:, None]
                rp -= g * dQ[j][1 + i]   # -div u
                ru[i] -= g * dQ[j][0]    # -d p / d x_i
        for f in range(4):
            own, nb = self.traces(Q, f)
            n = msh.normal[:, f]
            jp = nb[0] - own[0]
            jun = np.einsum("ikq,ki->kq", nb[1:] - own[1:], n)
            Fp = 0.5 * (self.tau_p * jp - jun)
            Fu = 0.5 * (self.tau_u * jun - jp)
            sc = msh.Fscale[:, f][:, None]
            rp += sc * (Fp @ self.Lf[f].T)
            lu = sc * (Fu @ self.Lf[f].T)
            for i in range(3):
                ru[i] += n[:, i][:, None] * lu
        if self.src is not None:
            rp += self.source_factor(t) * self.src
        if pre_wadg:
            return np.concatenate([rp[None], ru])
        if self.c2q is None:
            raise RuntimeError("c^2 not set")
        dp = (self.values_at_quad(rp) * self.c2q) @ self.Pq.T
        return np.concatenate([dp[None], ru])

    def step(self, Q, res, dt: float, nsteps: int, t0: float = 0.0):
        """Advance by nsteps low-storage RK4 steps from time t0; res is the 2N-storage
        register. Stage k of step n is evaluated at t0 + (n + c_k) dt."""
        Q = np.array(Q, dtype=np.float64)
        res = np.array(res, dtype=np.float64)
        for n in range(nsteps):
            for a, b, c in zip(LSRK4_A, LSRK4_B, LSRK4_C):
                R = self.rhs(Q, t=t0 + (n + c) * dt)
                res = a * res + dt * R
                Q = Q + b * res
        return Q, res

    # ------------------------------------------------------- energy quantities
    def inner(self, Q1, Q2):
        """Per-field sum_k J_k (q1, q2)_{ref} for state arrays [4, K, Np]."""
        return np.einsum("fki,ij,fkj,k->f", Q1, self.Mref, Q2, self.mesh.J)

    def face_dissipation(self, Q):
        """-(sum over faces) of the penalty terms: the exact value of sum_k (q, r(q)).

        Interior faces (each once): tau_p/2 [[p]]^2 + tau_u/2 ([[u]].n)^2; boundary
        faces: tau_p p^2 (p = 0 walls) or tau_u (u.n)^2 (rigid walls); integrals are
        over physical faces.
        """
        msh = self.mesh
        tot = 0.0
        for f in range(4):
            own, nb = self.traces(Q, f)
            n = msh.normal[:, f]
            jp = nb[0] - own[0]
            jun = np.einsum("ikq,ki->kq", nb[1:] - own[1:], n)
            integrand = 0.5 * self.tau_p * jp ** 2 + 0.5 * self.tau_u * jun ** 2
            wts = msh.Jf[:, f][:, None] * self.wf[None, :]
            per = np.sum(integrand * wts, axis=1)
            interior = ~self.bmask[f]
            # interior faces are visited from both sides: half each
            tot += 0.5 * np.sum(per[interior])
            bm = self.bmask[f]
            if self.bc == "p0":
                tot += np.sum(np.sum(self.tau_p * own[0, bm] ** 2 * wts[bm], axis=1))
            else:
                un = np.einsum("ikq,ki->kq", own[1:, bm], n[bm])
                tot += np.sum(np.sum(self.tau_u * un ** 2 * wts[bm], axis=1))
        return -tot

    def error_rule(self, nproj: int | None = None):
        """The rule of the error and energy integrals: collapsed Gauss-Jacobi with N+3 points
        per direction (exact to degree 2N+5), the rule of the degree-N projection. The paper
        does not fix the rule of its L^2 errors; this reading is shared with the library."""
        return tet_rule(self.N + 3 if nproj is None else nproj)

    def l2_error_sq(self, Q, fns, nproj: int | None = None):
        """Per-field sum_k J_k int_ref (q_h - f)^2 by the error rule, for a state Q [4, K, Np]
        (orthonormal coefficients) and four vectorised functions f(x, y, z)."""
        r, s, t, w = self.error_rule(nproj)
        vals = np.asarray(Q, dtype=np.float64) @ dubiner_tet(self.N, r, s, t).T  # [4, K, nq]
        X = self.mesh.map_points(r, s, t)
        ex = np.stack([np.broadcast_to(f(X[..., 0], X[..., 1], X[..., 2]), vals.shape[1:]) for f in fns])
        wJ = self.mesh.J[:, None] * w[None, :]
        return np.sum((vals - ex) ** 2 * wJ[None], axis=(1, 2))

    def energy_terms(self, Q, nproj: int | None = None):
        """(1/2) sum_k J_k int_ref of p^2 / c^2 and of u_i^2, by the error rule: [4] (the
        acoustic energy of eq. (awave) is their sum)."""
        r, s, t, w = self.error_rule(nproj)
        vals = np.asarray(Q, dtype=np.float64) @ dubiner_tet(self.N, r, s, t).T
        c2 = self.c2_at(r, s, t)
        wJ = 0.5 * self.mesh.J[:, None] * w[None, :]
        out = np.empty(4)
        out[0] = np.sum(vals[0] ** 2 / c2 * wJ)
        out[1:] = np.sum(vals[1:] ** 2 * wJ[None], axis=(1, 2))
        return out

    def energy(self, Q):
        """0.5 sum_k J_k (p^T W p + u^T M u), W = M M_{c^2}^{-1} M (weight-adjusted mass).

        Dense per-element solves; meant for small meshes."""
        if self.c2q is None:
            raise RuntimeError("c^2 not set")
        Q = np.asarray(Q, dtype=np.float64)
        E = 0.0
        Mc = np.einsum("qi,kq,qj->kij", self.Vq, self.c2q * self.wq[None, :], self.Vq)
        Mp = Q[0] @ self.Mref  # [K, Np]
        y = np.linalg.solve(Mc, Mp[..., None])[..., 0]
        E += np.sum(self.mesh.J * np.einsum("ki,ki->k", Mp, y))
        E += np.sum(self.inner(Q[1:], Q[1:]))
        return 0.5 * E
