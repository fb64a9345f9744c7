"""Pins of the oracle's receiver misfit gradient (``oracle/adjoint.py``): central finite
differences of the oracle's own forward misfit, which share nothing with the adjoint
recursion but the forward solve."""
import numpy as np
import pytest

from oracle import Oracle
from oracle.adjoint import Receivers, locate, misfit, misfit_gradient
from workloads import (c2_sinusoid, ic_gaussian_pulse, kuhn_cube_mesh, manufactured_source,
                       random_c2_coefficients, receiver_grid)


def _setup(n, N, M, bc, seed):
    xyz, etov = kuhn_cube_mesh(n)
    o = Oracle(xyz, etov, N, M, bc=bc)
    pulse = lambda x, y, z: ic_gaussian_pulse(x, y, z, centre=(0.4, 0.55, 0.5), width=0.2)  # noqa: E731
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    Q0 = o.project_initial([pulse, zero, zero, zero])
    c = random_c2_coefficients(seed, o.mesh.K, (M + 1) * (M + 2) * (M + 3) // 6)
    return xyz, etov, o, Q0, c


def test_locate_finds_containing_element():
    xyz, etov = kuhn_cube_mesh(2)
    o = Oracle(xyz, etov, 1, 0)
    pts = np.random.default_rng(3).uniform(0.0, 1.0, (40, 3))
    elem, rst = locate(o.mesh, pts)
    X = o.mesh.map_points(rst[:, 0], rst[:, 1], rst[:, 2])  # [K, npts, 3]
    assert np.allclose(X[elem, np.arange(40)], pts, atol=1e-13)
    lam = np.stack([-(1 + rst.sum(1)) / 2, (1 + rst[:, 0]) / 2, (1 + rst[:, 1]) / 2, (1 + rst[:, 2]) / 2], 1)
    assert np.all(lam >= -1e-10)
    with pytest.raises(ValueError):
        locate(o.mesh, [[1.5, 0.5, 0.5]])


@pytest.mark.parametrize("bc,M", [("rigid", 1), ("p0", 0)])
def test_gradient_matches_central_differences(bc, M):
    """6 tets, N = 2, 8 steps, 5 receivers; every coefficient of c checked."""
    xyz, etov, o, Q0, c = _setup(1, 2, M, bc, 21)
    rec = Receivers(o, [[0.3, 0.6, 1.0], [0.7, 0.2, 0.9], [0.5, 0.5, 0.5], [0.1, 0.8, 0.3], [0.9, 0.9, 0.05]])
    dt, nsteps = 0.02, 8
    target = random_c2_coefficients(22, *c.shape)
    o.set_c2_bernstein(target)
    data = misfit(o, Q0, dt, nsteps, rec, np.zeros((nsteps, 5)))[1]
    J, g, _ = misfit_gradient(o, c, Q0, dt, nsteps, rec, data)
    assert J > 0
    h = 1e-5
    fd = np.zeros_like(c)
    for idx in np.ndindex(*c.shape):
        cp, cm = c.copy(), c.copy()
        cp[idx] += h
        cm[idx] -= h
        o.set_c2_bernstein(cp)
        jp = misfit(o, Q0, dt, nsteps, rec, data)[0]
        o.set_c2_bernstein(cm)
        jm = misfit(o, Q0, dt, nsteps, rec, data)[0]
        fd[idx] = (jp - jm) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(fd)), (g, fd)


def test_gradient_with_source_matches_central_differences():
    """The source enters y = (B q)_p, so dJ/dc also carries Pi_N(dc^2 Pi_N f) terms."""
    xyz, etov, o, Q0, c = _setup(1, 2, 1, "p0", 23)
    o.set_source(manufactured_source(c2_sinusoid), amp=2.0, omega=np.pi)
    rec = Receivers(o, [[0.3, 0.6, 0.7], [0.5, 0.5, 0.5]])
    dt, nsteps = 0.02, 6
    data = np.zeros((nsteps, 2))
    J, g, _ = misfit_gradient(o, c, Q0, dt, nsteps, rec, data, t0=0.1)
    rng = np.random.default_rng(5)
    for _ in range(6):
        idx = (rng.integers(c.shape[0]), rng.integers(c.shape[1]))
        cp, cm = c.copy(), c.copy()
        cp[idx] += 1e-5
        cm[idx] -= 1e-5
        o.set_c2_bernstein(cp)
        jp = misfit(o, Q0, dt, nsteps, rec, data, t0=0.1)[0]
        o.set_c2_bernstein(cm)
        jm = misfit(o, Q0, dt, nsteps, rec, data, t0=0.1)[0]
        fd = (jp - jm) / 2e-5
        assert abs(g[idx] - fd) < 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (idx, g[idx], fd)


def test_zero_residual_gives_zero_gradient():
    xyz, etov, o, Q0, c = _setup(1, 1, 1, "rigid", 24)
    rec = Receivers(o, receiver_grid(2, 1.0))
    o.set_c2_bernstein(c)
    data = misfit(o, Q0, 0.02, 4, rec, np.zeros((4, 4)))[1]
    J, g, _ = misfit_gradient(o, c, Q0, 0.02, 4, rec, data)
    assert J == 0.0 and np.all(g == 0.0)


def test_receivers_sample_polynomials_exactly_at_any_point():
    """A projected polynomial of degree <= N is reproduced at the receivers, including mesh
    vertices (where the modal basis in collapsed coordinates is singular) and face points."""
    xyz, etov = kuhn_cube_mesh(2)
    o = Oracle(xyz, etov, 3, 0)
    f = lambda x, y, z: 1.0 + x - 2.0 * y * z + 0.5 * x ** 3  # noqa: E731
    Q = o.project_initial([f, f, f, f])
    pts = np.array([[0.5, 0.5, 0.5], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5, 0.0, 1.0], [0.25, 0.5, 0.75],
                    [0.3, 0.6, 1.0], [0.123, 0.456, 0.789]])
    rec = Receivers(o, pts)
    assert np.allclose(rec.sample(Q), f(pts[:, 0], pts[:, 1], pts[:, 2]), rtol=0, atol=1e-12)
