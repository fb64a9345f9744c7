"""Weight-adjusted update of the elastic velocity-stress system (test infrastructure only).

Paper Section 3.2, eq. (ewadg): the weighted mass matrices of rho v_t = ... and
C^{-1} sigma_t = ... are replaced by the weight-adjusted inverses M^{-1} M_{1/rho} and
(I (x) M^{-1}) M_C (I (x) M^{-1}); applied to the DG right-hand side r = (r_v, r_sigma) per
element this is, with isotropic C (Lame lambda, mu; Voigt order xx, yy, zz, yz, xz, xy),

    v'_i = P_q diag(1/rho) V_q r_v_i,
    sigma'_i = P_q [lambda tr(r_sigma) + 2 mu r_sigma_i](x_q)   (normal components),
    sigma'_s = P_q diag(mu) V_q r_sigma_s                        (shear components),

with V_q the modal basis at the oracle's volume rule (exact to degree 2N + M) and
P_q = M^{-1} V_q^T W, the weights being polynomials of degree M given by Bernstein
coefficients.
"""
from __future__ import annotations

import numpy as np

from .basis import bernstein_tet
from .wadg import Oracle


def weight_at_quad(o: Oracle, coef):
    """Bernstein coefficients [K, Mp] of degree M at the oracle's volume rule: [K, nq]."""
    return np.asarray(coef, dtype=np.float64) @ bernstein_tet(o.M, o.rq, o.sq, o.tq).T


def elastic_update(o: Oracle, R, rho_inv, lam, mu):
    """R: modal coefficients [9, K, Np] -> the weight-adjusted update, modal [9, K, Np]."""
    R = np.asarray(R, dtype=np.float64)
    wr, wl, wm = (weight_at_quad(o, c) for c in (rho_inv, lam, mu))
    V = R @ o.Vq.T  # [9, K, nq]
    tr = V[3] + V[4] + V[5]
    out = np.empty_like(V)
    for i in range(3):
        out[i] = wr * V[i]
        out[3 + i] = wl * tr + 2.0 * wm * V[3 + i]
        out[6 + i] = wm * V[6 + i]
    return out @ o.Pq.T


# The matrices A_i of the velocity-stress system (paper Section 3.2, eq. ewave), stress in the
# Voigt order xx, yy, zz, yz, xz, xy.
A_MATS = np.zeros((3, 6, 3))
A_MATS[0, 0, 0] = A_MATS[0, 4, 2] = A_MATS[0, 5, 1] = 1.0
A_MATS[1, 1, 1] = A_MATS[1, 3, 2] = A_MATS[1, 5, 0] = 1.0
A_MATS[2, 2, 2] = A_MATS[2, 3, 1] = A_MATS[2, 4, 0] = 1.0


def elastic_rhs(o: Oracle, Q, media=None, tau_v: float = 1.0, tau_s: float = 1.0, wall: str = "free"):
    """DG right-hand side of the velocity-stress system for the state Q [9, K, Np] (modal):

        r_v = sum_i A_i^T d sigma/dx_i + sum_f (J_f/J) L^f F_v,  F_v = A_n^T [[sigma]]/2 + tau_v A_n^T A_n [[v]]/2
        r_s = sum_i A_i  d v/dx_i      + sum_f (J_f/J) L^f F_s,  F_s = A_n [[v]]/2 + tau_s A_n A_n^T [[sigma]]/2

    with A_n = sum_i n_i A_i (the semi-discrete form after eq. ewave). Walls take mirror states:
    traction-free ("free") sigma+ = -sigma, v+ = v; rigid v+ = -v, sigma+ = sigma. With
    ``media`` = (1/rho, lambda, mu) Bernstein coefficients the weight-adjusted update follows
    (eq. ewadg); without, the pre-update right-hand side is returned."""
    Q = np.asarray(Q, dtype=np.float64)
    msh = o.mesh
    G = msh.G
    dQ = [Q @ Dj.T for Dj in o.D]
    dx = [sum(G[:, i, j][None, :, None] * dQ[j] for j in range(3)) for i in range(3)]  # d/dx_i, [9, K, Np]
    rv = np.zeros_like(Q[:3])
    rs = np.zeros_like(Q[3:])
    for i in range(3):
        rv += np.einsum("ba,bkn->akn", A_MATS[i], dx[i][3:])
        rs += np.einsum("ba,akn->bkn", A_MATS[i], dx[i][:3])
    for f in range(4):
        own = Q @ o.Vf[f].T
        nb = np.empty_like(own)
        for sel, ks2, Vn in o.groups[f]:
            nb[:, sel] = Q[:, ks2] @ Vn.T
        bm = o.bmask[f]
        if np.any(bm):
            if wall == "free":
                nb[:3, bm] = own[:3, bm]
                nb[3:, bm] = -own[3:, bm]
            else:
                nb[:3, bm] = -own[:3, bm]
                nb[3:, bm] = own[3:, bm]
        An = np.einsum("ki,ibc->kbc", msh.normal[:, f], A_MATS)  # [K, 6, 3]
        jv, js = nb[:3] - own[:3], nb[3:] - own[3:]
        AnT_js = np.einsum("kba,bkq->akq", An, js)
        An_jv = np.einsum("kba,akq->bkq", An, jv)
        Fv = 0.5 * AnT_js + 0.5 * tau_v * np.einsum("kba,bkq->akq", An, An_jv)
        Fs = 0.5 * An_jv + 0.5 * tau_s * np.einsum("kba,akq->bkq", An, AnT_js)
        sc = msh.Fscale[:, f][:, None]
        rv += sc * (Fv @ o.Lf[f].T)
        rs += sc * (Fs @ o.Lf[f].T)
    R = np.concatenate([rv, rs])
    if media is None:
        return R
    return elastic_update(o, R, *media)


def elastic_step(o: Oracle, Q, res, dt: float, nsteps: int, media, tau_v: float = 1.0, tau_s: float = 1.0,
                 wall: str = "free"):
    """nsteps of the 5-stage low-storage RK4 (the acoustic step's scheme) applied to the
    weighted elastic right-hand side: per stage res = a_k res + dt r(Q), Q = Q + b_k res.
    Q, res modal [9, K, Np]."""
    from .wadg import LSRK4_A, LSRK4_B
    Q = np.array(Q, dtype=np.float64)
    res = np.array(res, dtype=np.float64)
    for _ in range(nsteps):
        for a, b in zip(LSRK4_A, LSRK4_B):
            res = a * res + dt * elastic_rhs(o, Q, media, tau_v=tau_v, tau_s=tau_s, wall=wall)
            Q = Q + b * res
    return Q, res
