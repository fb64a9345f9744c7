"""Exact positivity check of the projected weight c^2_M (host side, no GPU).

The weight-adjusted scheme is energy stable for a positive weight (paper Section 3); the
library certifies c^2_M > 0 on the whole element from its Bernstein coefficients (they
bound the polynomial, Section 2) with edge bisection where they do not decide. These tests
build polynomials with known sign and compare against dense sampling with the oracle's own
Bernstein evaluator.
"""
import numpy as np
import pytest

from oracle.basis import bernstein_eval, bernstein_tet
from workloads import kuhn_cube_mesh


@pytest.fixture(scope="module")
def bb():
    from tests._build import ensure_built
    ensure_built()
    import paper_1808_08645_amd as bb
    return bb


def _ref_points(n_rand=20000, lattice=40, seed=0):
    """Reference-tetrahedron points: a degree-`lattice` barycentric lattice plus random points."""
    pts = []
    for i in range(lattice + 1):
        for j in range(lattice + 1 - i):
            for k in range(lattice + 1 - i - j):
                pts.append((i, j, k))
    lat = np.array(pts, float) / lattice  # lambda_1..3
    rng = np.random.default_rng(seed)
    lam = rng.dirichlet(np.ones(4), size=n_rand)[:, 1:]
    l123 = np.vstack([lat, lam])
    r, s, t = (2 * l123 - 1).T
    return r, s, t


def _phys_to_ref(verts, x):
    """Reference coordinates of physical points x [n,3] in the tet with vertices verts [4,3]
    (vertex 0 at r = s = t = -1, vertex i at the +1 end of coordinate i)."""
    A = np.stack([verts[1] - verts[0], verts[2] - verts[0], verts[3] - verts[0]], axis=1) / 2.0
    return np.linalg.solve(A, (x - verts[0]).T).T - 1.0


def test_positive_at_rule_points_but_negative_inside(bb):
    """c^2_M = |x - x0|^2 - delta (degree 2, projected exactly) is positive at every point of
    the projection rule but negative near x0: a rule-point check accepts it, the exact check
    rejects it, and the accepting policy stores it with the element counted."""
    xyz, etov = kuhn_cube_mesh(1)
    s = bb.Solver(xyz, etov, 3, 2, host_only=True)
    ev = s.element_vertices()
    x0 = xyz[ev[0]].mean(axis=0) + np.array([0.013, -0.007, 0.004])
    pts = s.projection_points(2)  # [K, nq, 3]
    d2min = float(np.min(np.sum((pts - x0) ** 2, axis=-1)))
    delta = 0.25 * d2min

    def f(x, y, z):
        return (x - x0[0]) ** 2 + (y - x0[1]) ** 2 + (z - x0[2]) ** 2 - delta

    samples = f(pts[..., 0], pts[..., 1], pts[..., 2])
    assert samples.min() > 0  # positive at every rule point
    coef = s.project_samples(2, samples)
    # the projection is exact for degree 2: f(x0) = -delta is reproduced
    r0 = _phys_to_ref(xyz[ev[0]], x0[None])[0]
    assert abs(bernstein_eval(2, coef[0], *r0)[0] + delta) < 1e-12
    with pytest.raises(bb.BBWADGError) as ei:
        s.set_c2(coef)
    assert ei.value.code == -3
    assert "not positive" in str(ei.value)
    nonpos, undecided, first = bb.bernstein_positivity(2, coef)
    assert (nonpos, undecided, first) == (1, 0, 0)
    s.set_c2_policy(True)
    s.set_c2(coef)
    assert s.c2_positivity() == (1, 0)
    s.set_c2_policy(False)
    with pytest.raises(bb.BBWADGError):
        s.set_c2(coef)
    assert bb.load_library().bbwadg_set_c2_policy(s._ctx, 7) == -1  # unknown policy


def test_positive_polynomial_with_negative_coefficients_is_accepted(bb):
    """(x - 1/2)^2 + 0.01 is positive everywhere although some Bernstein coefficients are
    negative: the subdivision has to decide it."""
    xyz, etov = kuhn_cube_mesh(1)
    s = bb.Solver(xyz, etov, 3, 2, host_only=True)
    coef = s.project_function(lambda x, y, z: (x - 0.5) ** 2 + 0.01, 2)
    assert coef.min() < 0
    s.set_c2(coef)
    assert s.c2_positivity() == (0, 0)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_classification_matches_dense_sampling(bb, m):
    """Random coefficient sets around 1: every set called positive has a positive minimum over
    ~30,000 sample points; every set called not positive has a sampled value <= 0 or within
    1e-3 of it (a negative region smaller than the sampling)."""
    rng = np.random.default_rng(100 + m)
    n = 300
    np_ = (m + 1) * (m + 2) * (m + 3) // 6
    coef = 1.0 + 0.9 * rng.standard_normal((n, np_))
    r, s_, t = _ref_points()
    vals = coef @ bernstein_tet(m, r, s_, t).T
    nonpos, undecided, _ = bb.bernstein_positivity(m, coef)
    assert undecided == 0
    # per-set classification through single-set calls
    cls = np.array([bb.bernstein_positivity(m, coef[i:i + 1])[0] for i in range(n)])
    assert cls.sum() == nonpos
    smin = vals.min(axis=1)
    assert np.all(smin[cls == 0] > 0)
    assert np.all(smin[cls == 1] < 1e-3)
    assert 0 < nonpos < n  # both outcomes occur


def test_vertex_value_zero_is_not_positive(bb):
    c = np.ones(10)
    c[0] = 0.0  # the value at vertex 0
    assert bb.bernstein_positivity(2, c)[0] == 1
    c[0] = 1e-300
    assert bb.bernstein_positivity(2, c)[0] == 0
    assert bb.bernstein_positivity(0, np.array([-1.0]))[0] == 1
    with pytest.raises(bb.BBWADGError) as ei:
        bb.bernstein_positivity(2, np.full(10, np.nan))
    assert ei.value.code == -3
