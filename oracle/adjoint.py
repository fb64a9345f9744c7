"""Receiver misfit and its gradient with respect to c^2_M (test infrastructure only).

The forward problem is the oracle's LSRK4 solve (quadrature WADG, paper Section 3.3 eq.
(pwadg), with the weight c^2_M given by per-element Bernstein coefficients c of degree M).
Receivers sample the pressure after every step, and the misfit is

    J(c) = 1/2 sum_{n=1..nsteps} sum_r (p(x_r, t_n) - d_{n,r})^2 .

Its gradient is taken by the plain discrete adjoint of the five-stage 2N-storage scheme:
with the stage map  r' = a_k r + dt A q,  q' = q + b_k r',  the transposed stage applied in
reverse order is

    v = rbar' + b_k qbar',   qbar = qbar' + dt A^T v,   rbar = a_k v,

and the c-dependence of A = W(c) B enters as  dJ/dc += dt v_p^T (dW/dc) y,  y = (B q)_p,
where W(c) is the per-element weighted projection P_q diag(c^2_M(x_q)) V_q on the pressure
field and B the DG operator before the weight adjustment (its pressure part includes the
source when one is set). A^T is formed from a dense matrix of B built column by column and
the explicit per-element matrices of W, all in the orthonormal modal basis, so this module
is only meant for meshes of a few dozen elements.
"""
from __future__ import annotations

import numpy as np

from .basis import bernstein_tet
from .wadg import LSRK4_A, LSRK4_B, LSRK4_C, Oracle


def locate(mesh, pts, tol: float = 1e-10):
    """Element and reference coordinates (r, s, t) of each physical point [npts, 3]: the
    lowest-numbered element whose barycentric coordinates are all >= -tol."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    elem = np.full(len(pts), -1, dtype=np.int64)
    rst = np.zeros((len(pts), 3))
    Ainv = np.linalg.inv(mesh.A)  # [K, 3, 3]: d r / d x
    v0 = mesh.verts[:, 0]
    for i, x in enumerate(pts):
        r = np.einsum("kij,kj->ki", Ainv, x[None, :] - v0) - 1.0
        lam = np.stack([-(1.0 + r.sum(1)) / 2.0, (1.0 + r[:, 0]) / 2.0, (1.0 + r[:, 1]) / 2.0,
                        (1.0 + r[:, 2]) / 2.0], axis=1)
        inside = np.nonzero(np.all(lam >= -tol, axis=1))[0]
        if len(inside) == 0:
            raise ValueError(f"point {x} is outside the mesh")
        elem[i] = inside[0]
        rst[i] = r[inside[0]]
    return elem, rst


class Receivers:
    """Pressure samples at fixed points: p(x_r) = sum_j Q_p[k_r, j] phi_j(r_r).

    The modal values phi are taken through the Bernstein basis, which is regular at every
    point of the element (the collapsed-coordinate form of the modal basis is singular at
    one vertex): phi(r) = B(r) T^{-1}, with T the exact Bernstein-to-modal change of basis."""

    def __init__(self, o: Oracle, pts):
        self.elem, self.rst = locate(o.mesh, pts)
        T = o.Pq @ bernstein_tet(o.N, o.rq, o.sq, o.tq)
        Bx = bernstein_tet(o.N, self.rst[:, 0], self.rst[:, 1], self.rst[:, 2])  # [nrec, Np]
        self.phi = Bx @ np.linalg.inv(T)

    def sample(self, Q):
        return np.einsum("rj,rj->r", Q[0, self.elem], self.phi)


def forward(o: Oracle, Q0, dt: float, nsteps: int, rec: Receivers, t0: float = 0.0, keep_stages=False):
    """Run nsteps LSRK4 steps from Q0 (modal, [4, K, Np]) recording the receivers after each
    step. Returns traces [nsteps, nrec] (and the input state of every stage if asked)."""
    Q = np.array(Q0, dtype=np.float64)
    res = np.zeros_like(Q)
    traces = np.zeros((nsteps, len(rec.elem)))
    stages = []
    for n in range(nsteps):
        for a, b, c in zip(LSRK4_A, LSRK4_B, LSRK4_C):
            if keep_stages:
                stages.append((Q.copy(), t0 + (n + c) * dt))
            res = a * res + dt * o.rhs(Q, t=t0 + (n + c) * dt)
            Q = Q + b * res
        traces[n] = rec.sample(Q)
    return (traces, stages) if keep_stages else traces


def misfit(o: Oracle, Q0, dt, nsteps, rec: Receivers, data, t0=0.0):
    tr = forward(o, Q0, dt, nsteps, rec, t0)
    return 0.5 * float(np.sum((tr - data) ** 2)), tr


def dg_operator_matrix(o: Oracle):
    """Dense matrix of the DG operator B before the weight adjustment (no source):
    column j is the pre-WADG right-hand side of the j-th unit state."""
    src = o.src
    o.src = None
    try:
        n = 4 * o.mesh.K * o.Np
        B = np.zeros((n, n))
        E = np.zeros(n)
        for j in range(n):
            E[j] = 1.0
            B[:, j] = o.rhs(E.reshape(4, o.mesh.K, o.Np), pre_wadg=True).ravel()
            E[j] = 0.0
    finally:
        o.src = src
    return B


def misfit_gradient(o: Oracle, c2_bern, Q0, dt: float, nsteps: int, rec: Receivers, data, t0: float = 0.0):
    """J and dJ/dc for the Bernstein coefficients c [K, Mp] of c^2_M. Returns (J, grad, traces)."""
    c2_bern = np.asarray(c2_bern, dtype=np.float64)
    o.set_c2_bernstein(c2_bern)
    K, Np = o.mesh.K, o.Np
    traces, stages = forward(o, Q0, dt, nsteps, rec, t0, keep_stages=True)
    resid = traces - data
    J = 0.5 * float(np.sum(resid ** 2))
    B = dg_operator_matrix(o)
    # per-element W_k = P_q diag(c^2_M(x_q)) V_q and the derivative tables T_g = P_q diag(B^M_g(x_q)) V_q
    W = np.einsum("iq,kq,qj->kij", o.Pq, o.c2q, o.Vq)
    BM = bernstein_tet(o.M, o.rq, o.sq, o.tq)  # [nq, Mp]
    T = np.einsum("iq,qg,qj->gij", o.Pq, BM, o.Vq)  # [Mp, Np, Np]
    grad = np.zeros((K, BM.shape[1]))
    lq = np.zeros((4, K, Np))
    lr = np.zeros((4, K, Np))
    for n in range(nsteps - 1, -1, -1):
        for i, k in enumerate(rec.elem):  # dJ/dq after step n
            lq[0, k] += resid[n, i] * rec.phi[i]
        for s in range(4, -1, -1):
            Qs, ts = stages[5 * n + s]
            v = lr + LSRK4_B[s] * lq
            y = o.rhs(Qs, pre_wadg=True, t=ts)[0]  # [K, Np]
            grad += dt * np.einsum("ki,gij,kj->kg", v[0], T, y)
            wv = v.copy()
            wv[0] = np.einsum("kij,ki->kj", W, v[0])  # W^T v on the pressure field
            lq = lq + dt * (B.T @ wv.ravel()).reshape(4, K, Np)
            lr = LSRK4_A[s] * v
    return J, grad, traces
