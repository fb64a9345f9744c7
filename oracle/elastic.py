"""Weight-adjusted update of the elastic velocity-stress system (test infrastructure only).

Paper Section 2.2, eq. (ewadg): the weighted mass matrices of rho v_t = ... and
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
