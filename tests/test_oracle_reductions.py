"""Pins of the oracle's FP64 reductions: the L^2 error against a reference solution and the
acoustic energy (1/2) int (p^2/c^2 + |u|^2) (no GPU, no HIP library).

Each is pinned to something other than itself: the mass-matrix norm (another rule and
another formula), exact reproduction of polynomials, the volume of the domain, the
weight-adjusted energy in the cases where the two energies coincide (constant c^2, and
p = c^2 g by the equality case of Cauchy-Schwarz) and the Cauchy-Schwarz bound otherwise.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.basis import dubiner_tet
from oracle.quadrature import tet_rule
from workloads import exact_sin_mode, kuhn_cube_mesh, random_c2_coefficients, random_state


def dimp(n):
    return (n + 1) * (n + 2) * (n + 3) // 6


REF_TET = (np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]]),
           np.array([[0, 1, 2, 3]], dtype=np.int64))


def _cube(N, M, n=2, seed=0):
    xyz, etov = kuhn_cube_mesh(n)
    o = Oracle(xyz, etov, N, M)
    Q = random_state(seed, o.mesh.K, o.Np)
    o.set_c2_bernstein(random_c2_coefficients(seed + 1, o.mesh.K, dimp(M)))
    return o, Q


@pytest.mark.parametrize("N", [1, 3, 5])
def test_error_against_zero_is_mass_norm(N):
    """||q - 0||^2 by the error rule equals sum_k J_k q^T M q (exact mass matrix)."""
    o, Q = _cube(N, 1)
    zero = [lambda x, y, z: 0.0 * x] * 4
    err = o.l2_error_sq(Q, zero)
    ref = o.inner(Q, Q)
    assert np.allclose(err, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("N", [2, 4])
def test_error_against_itself_vanishes(N):
    """On the reference element (x = r) a polynomial state has zero error against itself."""
    xyz, etov = REF_TET
    o = Oracle(xyz, etov, N, 0)
    Q = random_state(3, 1, o.Np)
    fns = [lambda x, y, z, f=f: dubiner_tet(N, x.ravel(), y.ravel(), z.ravel()).reshape(x.shape + (-1,)) @ Q[f, 0]
           for f in range(4)]
    err = o.l2_error_sq(Q, fns)
    assert np.all(err < 1e-26 * max(1.0, np.abs(o.inner(Q, Q)).max()))


def test_error_of_constant_is_volume():
    """q = 0 against f = a: a^2 times the volume of the unit cube."""
    o, Q = _cube(3, 1)
    consts = [0.5, -2.0, 3.0, 1.25]
    fns = [lambda x, y, z, a=a: a + 0.0 * x for a in consts]
    err = o.l2_error_sq(np.zeros_like(Q), fns)
    assert np.allclose(err, np.square(consts), rtol=1e-13)


def test_error_of_standing_wave_converges():
    """Projected standing wave: the error falls like h^{N+1} (N = 2, h = 1/2 -> 1/4)."""
    errs = []
    for n in (2, 4):
        xyz, etov = kuhn_cube_mesh(n)
        o = Oracle(xyz, etov, 2, 0)
        fns = [lambda x, y, z, i=i: exact_sin_mode(x, y, z, 0.3)[i] for i in range(4)]
        Q = o.project_initial(fns)
        errs.append(np.sqrt(o.l2_error_sq(Q, fns).sum()))
    assert np.log2(errs[0] / errs[1]) > 2.5, errs


@pytest.mark.parametrize("N", [2, 4])
def test_energy_constant_c_equals_weight_adjusted(N):
    """c^2 = c0: (1/2) int p^2/c0 + |u|^2 is the weight-adjusted energy, W = M/c0."""
    o, Q = _cube(N, 1)
    o.set_c2_bernstein(np.full((o.mesh.K, 4), 1.75))
    e = o.energy_terms(Q)
    assert np.isclose(e.sum(), o.energy(Q), rtol=1e-12)
    assert np.allclose(e[0], 0.5 * o.inner(Q, Q)[0] / 1.75, rtol=1e-12)
    assert np.allclose(e[1:], 0.5 * o.inner(Q, Q)[1:], rtol=1e-12)


@pytest.mark.parametrize("N,M", [(2, 1), (4, 1), (4, 2)])
def test_energy_equality_case_p_is_c2_times_polynomial(N, M):
    """p = c^2 g with deg c^2 + deg g <= N: p^T M M_c^{-1} M p = int c^2 g^2 = int p^2/c^2.

    Cauchy-Schwarz in the c^2-weighted inner product is an equality for v = g in P^N."""
    xyz, etov = REF_TET
    o = Oracle(xyz, etov, N, M)
    rng = np.random.default_rng(7)
    ca = rng.uniform(0.2, 0.5, size=(M + 1, 3))

    def c2(x, y, z):  # degree M, between 1 and 4 on the element
        v = 2.5 + 0.0 * x
        for d in range(1, M + 1):
            v = v + ca[d, 0] * x ** d + ca[d, 1] * y ** d + ca[d, 2] * z ** d
        return v
    gdeg = N - M
    gc = rng.standard_normal(dimp(gdeg))

    def g(x, y, z):
        return dubiner_tet(gdeg, x.ravel(), y.ravel(), z.ravel()).reshape(x.shape + (-1,)) @ gc

    o.set_c2_function(c2, project=True)
    p = o.project_modal(lambda x, y, z: c2(x, y, z) * g(x, y, z), N)
    Q = np.zeros((4, 1, o.Np))
    Q[0] = p
    r, s, t, w = tet_rule(N + M + 4)  # exact for c^2 g^2
    direct = 0.5 * np.sum(w * c2(r, s, t) * g(r, s, t) ** 2)
    e = o.energy_terms(Q)
    assert np.isclose(e[0], direct, rtol=1e-12)
    assert np.isclose(o.energy(Q), direct, rtol=1e-12)


@pytest.mark.parametrize("N,M", [(3, 1), (5, 2)])
def test_energy_bounds_weight_adjusted_energy(N, M):
    """Variable c^2: the weight-adjusted energy is at most (1/2) int p^2/c^2 + |u|^2."""
    o, Q = _cube(N, M, seed=4)
    e = o.energy_terms(Q)
    w = o.energy(Q)
    assert w <= e.sum() * (1 + 1e-12)
    assert w >= 0.5 * e.sum()  # same order: c^2 in [0.5, 2]
