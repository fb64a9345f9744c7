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


def test_elastic_rhs_conserves_energy_with_central_fluxes():
    """With tau = 0 and either wall type, sum_k (Q, r(Q))_{L^2} = 0: the volume terms and the
    central fluxes form a skew operator (a wrong sign or a transposed A_i breaks this)."""
    from oracle.elastic import elastic_rhs
    xyz, etov = kuhn_cube_mesh(2)
    o = Oracle(xyz, etov, 3, 0)
    Q = np.random.default_rng(7).standard_normal((9, o.mesh.K, o.Np))
    J = o.mesh.J[None, :, None]
    for wall in ("free", "rigid"):
        R = elastic_rhs(o, Q, tau_v=0.0, tau_s=0.0, wall=wall)
        e = np.sum(J * Q * R)
        assert abs(e) < 1e-11 * np.sum(J * np.abs(Q) * np.abs(R)), (wall, e)
        R = elastic_rhs(o, Q, tau_v=1.0, tau_s=0.7, wall=wall)
        assert np.sum(J * Q * R) < 0  # the penalty terms dissipate


def test_elastic_rhs_of_a_global_polynomial_on_interior_elements():
    """On elements away from the walls the traces agree, so r is the exact derivative term:
    r_v = div sigma and r_s = the symmetric gradient of v (Voigt, shear entries doubled)."""
    from oracle.elastic import elastic_rhs
    xyz, etov = kuhn_cube_mesh(3)
    o = Oracle(xyz, etov, 3, 0)
    v = [lambda x, y, z: x * y + z, lambda x, y, z: z * z - x, lambda x, y, z: x * y * z]
    s = [lambda x, y, z: x * x, lambda x, y, z: y * z, lambda x, y, z: x - y * y * z,
         lambda x, y, z: x * z, lambda x, y, z: y + z * x * x, lambda x, y, z: x * y]
    Q = np.stack([o.project_modal(f, o.N) for f in v + s])
    R = elastic_rhs(o, Q, tau_v=1.0, tau_s=1.0)
    inner = np.all(o.mesh.nbr >= 0, axis=1)
    X = o.mesh.map_points(o.rq, o.sq, o.tq)
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    # sxx = x^2, syy = yz, szz = x - y^2 z, syz = xz, sxz = y + z x^2, sxy = xy
    want = np.stack([
        2 * x + x + x * x,       # d sxx/dx + d sxy/dy + d sxz/dz
        y + z + x,               # d sxy/dx + d syy/dy + d syz/dz
        2 * x * z - y * y,       # d sxz/dx + d syz/dy + d szz/dz
        y,                       # d v1/dx
        0 * x,                   # d v2/dy
        x * y,                   # d v3/dz
        x * z + 2 * z,           # d v3/dy + d v2/dz
        y * z + 1.0,             # d v3/dx + d v1/dz
        x - 1.0,                 # d v2/dx + d v1/dy
    ])
    got = o.values_at_quad(R)
    assert np.max(np.abs(got[:, inner] - want[:, inner])) < 1e-10


def test_elastic_step_is_fourth_order_against_the_matrix_exponential():
    """One oracle step against exp(dt L) Q, with L the assembled weighted right-hand side on a
    6-tet mesh (brute force, scipy's expm): the local error falls by about 2^5 when dt halves,
    as a 4th-order scheme's must (a dropped or mis-weighted stage lowers the order)."""
    from scipy.linalg import expm
    from oracle.elastic import elastic_rhs, elastic_step
    xyz, etov = kuhn_cube_mesh(1)
    o = Oracle(xyz, etov, 1, 0)
    K, Np = o.mesh.K, o.Np
    media = _media(K, 1, 3)
    n = 9 * K * Np
    L = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        L[:, j] = elastic_rhs(o, e.reshape(9, K, Np), media, tau_v=1.0, tau_s=1.0, wall="rigid").ravel()
    Q = np.random.default_rng(5).standard_normal((9, K, Np))
    rho = np.abs(np.linalg.eigvals(L)).max()
    errs = []
    for dt in (0.4 / rho, 0.2 / rho):
        Q1, _ = elastic_step(o, Q, np.zeros_like(Q), dt, 1, media, wall="rigid")
        errs.append(np.linalg.norm(Q1.ravel() - expm(dt * L) @ Q.ravel()))
    ratio = errs[0] / errs[1]
    assert 24.0 < ratio < 40.0, (errs, ratio)
