"""Pins of the elastic weight-adjusted update oracle (``oracle/elastic.py``) against what
the mathematics fixes: Hooke's law for constant media, exactness when the products stay in
P^N, and the symmetry of the matrix-weighted projection for a symmetric C."""
import numpy as np

from oracle import Oracle
from oracle.elastic import elastic_update
from workloads import kuhn_cube_mesh


def _media(K, Mp, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.5, 1.5, (K, Mp)), rng.uniform(0.5, 2.0, (K, Mp)), rng.uniform(0.3, 1.0, (K, Mp)))


def test_constant_media_apply_hookes_law():
    xyz, etov = kuhn_cube_mesh(1)
    o = Oracle(xyz, etov, 3, 2)
    K, Np, Mp = o.mesh.K, o.Np, 10
    R = np.random.default_rng(1).standard_normal((9, K, Np))
    rho_inv, lam, mu = 0.7, 1.9, 0.45
    out = elastic_update(o, R, np.full((K, Mp), rho_inv), np.full((K, Mp), lam), np.full((K, Mp), mu))
    tr = R[3] + R[4] + R[5]
    want = np.concatenate([rho_inv * R[:3], lam * tr[None] + 2 * mu * R[3:6], mu * R[6:]])
    assert np.allclose(out, want, rtol=0, atol=1e-12)


def test_exact_when_products_stay_in_PN():
    """deg(weights) + deg(r) <= N: the update equals the pointwise product (no projection error)."""
    xyz, etov = kuhn_cube_mesh(1)
    N, M = 4, 2
    o = Oracle(xyz, etov, N, M)
    K = o.mesh.K
    rng = np.random.default_rng(2)
    rho_inv, lam, mu = _media(K, 10, 3)
    # random fields of degree N - M, written in the degree-N modal basis (higher modes zero)
    Rlow = o.project_initial([lambda x, y, z, a=a: a[0] + a[1] * x * y + a[2] * z * z - a[3] * x
                              for a in rng.standard_normal((4, 4))])
    R = np.concatenate([Rlow, Rlow[:3] * 0.5, Rlow[1:3]], axis=0)  # 9 fields of degree 2
    out = elastic_update(o, R, rho_inv, lam, mu)
    from oracle.elastic import weight_at_quad
    V = R @ o.Vq.T
    wr, wl, wm = (weight_at_quad(o, c) for c in (rho_inv, lam, mu))
    tr = V[3] + V[4] + V[5]
    want = np.concatenate([wr * V[:3], wl * tr + 2 * wm * V[3:6], wm * V[6:]])
    assert np.max(np.abs(out @ o.Vq.T - want)) < 1e-11 * np.max(np.abs(want))


def test_matrix_weighted_projection_is_symmetric():
    """(W r1, r2) = (r1, W r2) in L^2 (orthonormal modal basis, per element) for symmetric C."""
    xyz, etov = kuhn_cube_mesh(1)
    o = Oracle(xyz, etov, 3, 1)
    K, Np = o.mesh.K, o.Np
    rng = np.random.default_rng(4)
    rho_inv, lam, mu = _media(K, 4, 5)
    R1, R2 = rng.standard_normal((2, 9, K, Np))
    a = np.sum(elastic_update(o, R1, rho_inv, lam, mu) * R2)
    b = np.sum(R1 * elastic_update(o, R2, rho_inv, lam, mu))
    assert abs(a - b) < 1e-12 * (abs(a) + 1.0)
    # and positive for positive media (lambda, mu > 0): (W r, r) > 0
    assert np.sum(elastic_update(o, R1, rho_inv, lam, mu) * R1) > 0
