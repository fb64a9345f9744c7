"""Pins of the CPU oracle against what the mathematics fixes (no GPU, no HIP library).

Each test checks the oracle against something other than itself: library routines,
closed-form integrals, exact polynomial reproduction, the exact semi-discrete energy
identity, the constant-c reduction (paper Section 3.1), exact solutions and convergence
rates, and the Runge-Kutta order conditions.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest
from scipy.special import roots_jacobi

from oracle import Oracle
from oracle.basis import bernstein_tet, dubiner_tet, multi_indices
from oracle.mesh import Mesh
from oracle.quadrature import gauss_jacobi, tet_rule, tri_rule
from oracle.wadg import LSRK4_A, LSRK4_B, LSRK4_C
from workloads import (exact_cos_mode, exact_sin_mode, kuhn_cube_mesh, random_c2_coefficients,
                       random_state)


def dimp(n):
    return (n + 1) * (n + 2) * (n + 3) // 6


# ------------------------------------------------------------------ quadrature
@pytest.mark.parametrize("n,a,b", [(1, 0, 0), (4, 0, 0), (7, 1, 0), (9, 2, 0), (12, 2, 0)])
def test_gauss_jacobi_matches_library(n, a, b):
    x, w = gauss_jacobi(n, a, b)
    xr, wr = roots_jacobi(n, a, b)
    assert np.allclose(np.sort(x), np.sort(xr), atol=1e-13)
    assert np.allclose(w[np.argsort(x)], wr[np.argsort(xr)], rtol=1e-12)


@pytest.mark.parametrize("n", [1, 3, 6, 9])
def test_tet_rule_integrates_barycentric_monomials(n):
    """Dirichlet integral: int_T lambda^alpha = |T| 3! alpha! / (|alpha| + 3)!."""
    r, s, t, w = tet_rule(n)
    lam = np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2])
    assert abs(w.sum() - 4.0 / 3.0) < 1e-14
    rng = np.random.default_rng(0)
    for _ in range(20):
        deg = int(rng.integers(0, 2 * n))
        cut = np.sort(rng.integers(0, deg + 1, size=3))
        al = np.diff(np.concatenate([[0], cut, [deg]]))
        exact = 4.0 / 3.0 * 6 * np.prod([factorial(int(x)) for x in al]) / factorial(deg + 3)
        val = np.sum(w * np.prod([lam[j] ** al[j] for j in range(4)], axis=0))
        assert abs(val - exact) <= 1e-13 * max(1.0, exact)


@pytest.mark.parametrize("n", [1, 4, 8])
def test_tri_rule_integrates_barycentric_monomials(n):
    r, s, w = tri_rule(n)
    mu = np.stack([-(r + s) / 2, (1 + r) / 2, (1 + s) / 2])
    assert abs(w.sum() - 2.0) < 1e-14
    for al in [(0, 0, 0), (1, 0, 0), (2, 1, 0), (n, n - 1, 0), (n - 1, 0, n)]:
        deg = sum(al)
        if deg > 2 * n - 1:
            continue
        exact = 2.0 * 2 * np.prod([factorial(x) for x in al]) / factorial(deg + 2)
        val = np.sum(w * np.prod([mu[j] ** al[j] for j in range(3)], axis=0))
        assert abs(val - exact) < 1e-13


# ---------------------------------------------------------------------- bases
@pytest.mark.parametrize("N", [1, 3, 5, 9])
def test_dubiner_is_orthonormal(N):
    r, s, t, w = tet_rule(N + 1)
    V = dubiner_tet(N, r, s, t)
    assert np.abs(V.T @ (w[:, None] * V) - np.eye(dimp(N))).max() < 1e-12


@pytest.mark.parametrize("N", [2, 5, 9])
def test_dubiner_gradient_matches_finite_differences(N):
    rng = np.random.default_rng(N)
    lam = rng.dirichlet(np.ones(4), size=5).T
    r, s, t = 2 * lam[1] - 1, 2 * lam[2] - 1, 2 * lam[3] - 1
    V, G = dubiner_tet(N, r, s, t, grad=True)
    h = 1e-6
    for d, (dr, ds, dt) in enumerate([(h, 0, 0), (0, h, 0), (0, 0, h)]):
        fd = (dubiner_tet(N, r + dr, s + ds, t + dt) - dubiner_tet(N, r - dr, s - ds, t - dt)) / (2 * h)
        assert np.abs(fd - G[d]).max() < 1e-6 * max(1.0, np.abs(G[d]).max())


@pytest.mark.parametrize("N", [1, 4, 7])
def test_bernstein_partition_of_unity_and_vertices(N):
    rng = np.random.default_rng(1)
    lam = rng.dirichlet(np.ones(4), size=9).T
    B = bernstein_tet(N, 2 * lam[1] - 1, 2 * lam[2] - 1, 2 * lam[3] - 1)
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-14)
    # at vertex j only the coefficient N e_j survives
    verts = [(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]
    mis = multi_indices(N)
    for j, v in enumerate(verts):
        Bv = bernstein_tet(N, *[np.array([x], float) for x in v])[0]
        e = [0, 0, 0, 0]
        e[j] = N
        assert np.isclose(Bv[mis.index(tuple(e))], 1.0) and np.isclose(Bv.sum(), 1.0)


# --------------------------------------------------------------------- mesh
@pytest.mark.parametrize("n", [1, 3])
def test_kuhn_mesh_geometry(n):
    xyz, etov = kuhn_cube_mesh(n)
    m = Mesh(xyz, etov)
    assert m.K == 6 * n ** 3
    assert abs(np.sum(m.J) * 4.0 / 3.0 - 1.0) < 1e-13  # total volume 1
    nb = np.sum(m.nbr < 0)
    assert nb == 12 * n * n  # each cube face split into two triangles
    # closed surface: sum_f |f| n_f = 0 for every element
    s = np.einsum("kf,kfi->ki", m.area, m.normal)
    assert np.abs(s).max() < 1e-14
    # G is the inverse of dx/dr
    I = np.einsum("kij,kjl->kil", m.A, np.transpose(m.G, (0, 2, 1)))
    assert np.abs(I - np.eye(3)).max() < 1e-12
    # neighbour symmetry
    for k in range(m.K):
        for f in range(4):
            k2, f2 = m.nbr[k, f], m.nbr_face[k, f]
            if k2 >= 0:
                assert m.nbr[k2, f2] == k and m.nbr_face[k2, f2] == f
                assert np.allclose(m.normal[k, f], -m.normal[k2, f2])


# -------------------------------------------------------------- DG operators
def _setup(N, M, bc="p0", tau=(1.0, 1.0), n=2, seed=0):
    xyz, etov = kuhn_cube_mesh(n)
    o = Oracle(xyz, etov, N, M, tau_p=tau[0], tau_u=tau[1], bc=bc)
    Q = random_state(seed, o.mesh.K, o.Np)
    o.set_c2_bernstein(random_c2_coefficients(seed + 1, o.mesh.K, dimp(M)))
    return o, Q


@pytest.mark.parametrize("N,M", [(1, 0), (2, 1), (3, 1), (4, 2), (6, 3)])
@pytest.mark.parametrize("bc", ["p0", "rigid"])
@pytest.mark.parametrize("tau", [(1.0, 1.0), (0.0, 0.0), (0.5, 2.0)])
def test_semidiscrete_energy_identity(N, M, bc, tau):
    """sum_k [(p, r_p) + (u, r_u)] equals minus the penalty face terms, for any state.

    Integrating by parts element-wise, the volume terms cancel against the average parts
    of the fluxes and what is left is the jump penalty on interior faces and the mirror-
    state penalty on boundary faces; it is zero for tau = 0.
    """
    o, Q = _setup(N, M, bc, tau)
    lhs = o.inner(Q, o.rhs(Q, pre_wadg=True)).sum()
    rhs = o.face_dissipation(Q)
    scale = max(1.0, abs(rhs), np.abs(o.inner(Q, Q)).sum())
    assert abs(lhs - rhs) < 1e-12 * scale


def _bernstein_product_integrals(N, M, c2):
    """Reference-element integrals of Bernstein products in closed form, without quadrature:
    int B^N_a B^N_b = |T| 3! (N!)^2 / (2N+3)! (a+b)!/(a! b!) and
    int B^N_a B^N_b B^M_g = |T| 3! (N!)^2 M! / (2N+M+3)! (a+b+g)!/(a! b! g!)
    (multi-index factorials over the four barycentric components; the factor |T| 3! is left
    out, it is common to both). Returns the mass matrix [Np, Np] and the c^2-weighted mass
    matrices [K, Np, Np] for Bernstein coefficients c2 [K, Mp] of degree M."""
    A, G = multi_indices(N), multi_indices(M)

    def mf(k):
        return float(np.prod([factorial(x) for x in k]))

    def add(*ks):
        return tuple(sum(v) for v in zip(*ks))

    Mb = np.array([[mf(add(a, b)) / (mf(a) * mf(b)) for b in A] for a in A])
    Mb *= factorial(N) ** 2 / factorial(2 * N + 3)
    T3 = np.array([[[mf(add(a, b, g)) / (mf(a) * mf(b) * mf(g)) for g in G] for b in A] for a in A])
    T3 *= factorial(N) ** 2 * factorial(M) / factorial(2 * N + M + 3)
    return Mb, np.einsum("abg,kg->kab", T3, c2)


@pytest.mark.parametrize("N,M", [(2, 1), (4, 2), (5, 2), (3, 3)])
def test_weight_adjusted_step_against_closed_form_bernstein_integrals(N, M):
    """W dp/dt = M r_p with W = M M_{c^2}^{-1} M, i.e. M dp = M_{c^2} r_p: the oracle's step
    (orthonormal basis, quadrature) against both mass matrices written out in the Bernstein
    basis from the closed-form simplex integrals of Bernstein products. A rule not exact to
    degree 2N+M, c^2 taken at the wrong points or a wrong projection all break it."""
    o, Q = _setup(N, M)
    c2 = random_c2_coefficients(1, o.mesh.K, dimp(M))  # the weight _setup installs
    pre = o.rhs(Q, pre_wadg=True)[0]
    dp = o.rhs(Q)[0]
    to_bern = np.linalg.inv(o.from_bernstein(np.eye(o.Np)))  # orthonormal -> Bernstein (rows)
    pre_b, dp_b = pre @ to_bern, dp @ to_bern
    Mb, Mc = _bernstein_product_integrals(N, M, c2)
    lhs = dp_b @ Mb  # Mb is symmetric
    rhs = np.einsum("kab,kb->ka", Mc, pre_b)
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(rhs).max()
    # the check sees the weight: one Bernstein coefficient of c^2 dropped breaks it
    c2_drop = c2.copy()
    c2_drop[:, -1] = 0.0
    rhs_drop = np.einsum("kab,kb->ka", _bernstein_product_integrals(N, M, c2_drop)[1], pre_b)
    assert np.abs(lhs - rhs_drop).max() > 1e-4 * np.abs(rhs).max()


@pytest.mark.parametrize("N", [2, 4])
def test_constant_c_reduces_to_scaled_dg(N):
    """For c^2 = c0 constant the weight-adjusted inverse is c0 M^{-1} (paper Section 3.1)."""
    o, Q = _setup(N, 1)
    o.set_c2_bernstein(np.full((o.mesh.K, 4), 2.5))  # constant in Bernstein form
    pre = o.rhs(Q, pre_wadg=True)
    full = o.rhs(Q)
    assert np.abs(full[0] - 2.5 * pre[0]).max() < 1e-12 * np.abs(pre[0]).max()
    assert np.array_equal(full[1:], pre[1:])


@pytest.mark.parametrize("N", [1, 3, 5])
def test_exact_derivative_of_global_polynomials(N):
    """For globally continuous polynomial states of degree <= N all jumps vanish, so
    r_u = -grad p (rigid walls, u = 0) and r_p = -div u (p = 0 walls, p = 0) exactly."""
    xyz, etov = kuhn_cube_mesh(2)
    rng = np.random.default_rng(7)
    cp = rng.normal(size=(N + 1, N + 1, N + 1))
    exps = [(a, b, c) for a in range(N + 1) for b in range(N + 1) for c in range(N + 1) if a + b + c <= N]

    def poly(x, y, z, dx=None):
        out = np.zeros_like(x)
        for (a, b, c) in exps:
            e = [a, b, c]
            coef = cp[a, b, c]
            if dx is not None:
                if e[dx] == 0:
                    continue
                coef = coef * e[dx]
                e[dx] -= 1
            out = out + coef * x ** e[0] * y ** e[1] * z ** e[2]
        return out

    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    o = Oracle(xyz, etov, N, 0, bc="rigid")
    Q = o.project_initial([poly, zero, zero, zero])
    R = o.rhs(Q, pre_wadg=True)
    X = o.mesh.map_points(o.rq, o.sq, o.tq)
    vals = o.values_at_quad(R)
    for i in range(3):
        ex = -poly(X[..., 0], X[..., 1], X[..., 2], dx=i)
        assert np.abs(vals[1 + i] - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())
    assert np.abs(vals[0]).max() < 1e-10
    o2 = Oracle(xyz, etov, N, 0, bc="p0")
    Q2 = o2.project_initial([zero, poly, poly, poly])
    R2 = o2.values_at_quad(o2.rhs(Q2, pre_wadg=True))
    ex = -sum(poly(X[..., 0], X[..., 1], X[..., 2], dx=i) for i in range(3))
    assert np.abs(R2[0] - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())


def test_bernstein_to_modal_roundtrip_is_exact():
    o, _ = _setup(4, 2)
    bern = random_state(3, o.mesh.K, o.Np)
    Q = o.from_bernstein(bern)
    assert np.abs(o.values_at_quad(Q) - o.bernstein_values_at_quad(bern)).max() < 1e-12


def test_c2_projection_reproduces_polynomials():
    """The per-element L^2 projection onto P^M is the identity on P^M."""
    o, _ = _setup(3, 2)
    f = lambda x, y, z: 1.0 + 0.3 * x - 0.2 * y * z + 0.7 * z * z  # noqa: E731
    o.set_c2_function(f, project=True)
    X = o.mesh.map_points(o.rq, o.sq, o.tq)
    assert np.abs(o.c2q - f(X[..., 0], X[..., 1], X[..., 2])).max() < 1e-13


# ---------------------------------------------------------------- time stepping
def test_lsrk4_stability_polynomial():
    """Applied to y' = z y the scheme gives R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200.

    Computed in exact rational arithmetic from the (rational) coefficients."""
    A = [Fraction(x).limit_denominator(10 ** 14) for x in LSRK4_A]
    B = [Fraction(x).limit_denominator(10 ** 14) for x in LSRK4_B]

    L = 8  # polynomials in z, truncated past z^7 (the scheme has 5 stages)
    y = [Fraction(1)] + [Fraction(0)] * (L - 1)
    res = [Fraction(0)] * L
    for a, b in zip(A, B):
        zy = [Fraction(0)] + y[:-1]
        res = [a * r + v for r, v in zip(res, zy)]
        y = [yy + b * rr for yy, rr in zip(y, res)]
    coeffs = [float(c) for c in y[:6]]
    expect = [1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 200]
    assert np.allclose(coeffs[:5], expect[:5], rtol=0, atol=1e-12)
    assert abs(coeffs[5] - 1 / 200) < 1e-4


def test_lsrk4_fourth_order_on_nonlinear_ode():
    """y' = -y^2 + sin(t), integrated with stage times c_k; the error falls as dt^4."""
    def run(nsteps):
        dt = 1.0 / nsteps
        y, res, t = 1.0, 0.0, 0.0
        for _ in range(nsteps):
            for a, b, c in zip(LSRK4_A, LSRK4_B, LSRK4_C):
                res = a * res + dt * (-y * y + np.sin(t + c * dt))
                y = y + b * res
            t += dt
        return y
    ref = run(4096)
    e1, e2 = abs(run(16) - ref), abs(run(32) - ref)
    rate = np.log2(e1 / e2)
    assert 3.7 < rate < 4.4


def test_lsrk4_stage_times_consistent():
    """c_k is the time reached after stage k-1: c_{k+1} = sum over earlier stages."""
    # For a 2N-storage scheme the stage time is the integral of y' = 1 after the stage.
    y, res = 0.0, 0.0
    cs = []
    for a, b in zip(LSRK4_A, LSRK4_B):
        cs.append(y)
        res = a * res + 1.0
        y = y + b * res
    assert np.allclose(cs, LSRK4_C, atol=1e-12)
    assert abs(y - 1.0) < 1e-12


@pytest.mark.parametrize("bc,exact", [("p0", exact_sin_mode), ("rigid", exact_cos_mode)])
def test_standing_wave_convergence_rate(bc, exact):
    """c = 1 standing waves on the unit cube: L^2 error falls like h^{N+1}."""
    N, T = 2, 0.1
    errs = []
    for n in (2, 4):
        xyz, etov = kuhn_cube_mesh(n)
        o = Oracle(xyz, etov, N, 0, bc=bc)
        o.set_c2_bernstein(np.ones((o.mesh.K, 1)))
        fns = [lambda x, y, z, i=i: exact(x, y, z, 0.0)[i] for i in range(4)]
        Q = o.project_initial(fns)
        nsteps = 40
        Q, _ = o.step(Q, np.zeros_like(Q), T / nsteps, nsteps)
        X = o.mesh.map_points(o.rq, o.sq, o.tq)
        ex = np.stack(exact(X[..., 0], X[..., 1], X[..., 2], T))
        err = np.sqrt(o.l2_sq(o.values_at_quad(Q) - ex).sum())
        errs.append(err)
    rate = np.log2(errs[0] / errs[1])
    assert rate > N + 1 - 0.5, (errs, rate)


def test_energy_nonincreasing_cube384_config():
    """Fully discrete: the weight-adjusted energy does not grow over 10 steps at CFL 0.5."""
    from workloads import c2_sinusoid, ic_cos_product
    xyz, etov = kuhn_cube_mesh(4)
    o = Oracle(xyz, etov, 3, 1, bc="p0")
    o.set_c2_function(c2_sinusoid, project=True)
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    Q = o.project_initial([ic_cos_product, zero, zero, zero])
    res = np.zeros_like(Q)
    dt = 0.5 * 0.25 / (np.sqrt(1.5) * 16.0)
    E = [o.energy(Q)]
    for _ in range(10):
        Q, res = o.step(Q, res, dt, 1)
        E.append(o.energy(Q))
    assert all(E[i + 1] <= E[i] * (1 + 1e-13) for i in range(10)), E


# ------------------------------------------------------------------ manufactured source
def test_source_enters_linearly_in_time():
    """With Q = 0 the right-hand side is the source alone: dp/dt = s(t) Pi_N(c^2 Pi_N g),
    du/dt = 0, with s(t) = amp sin(omega t + phase)."""
    from workloads import c2_sinusoid, manufactured_source
    xyz, etov = kuhn_cube_mesh(2)
    o = Oracle(xyz, etov, 3, 1)
    o.set_c2_function(c2_sinusoid, project=True)
    o.set_source(manufactured_source(c2_sinusoid), amp=1.7, omega=2.0, phase=0.3)
    Z = np.zeros((4, o.mesh.K, o.Np))
    r1 = o.rhs(Z, t=0.1)
    r2 = o.rhs(Z, t=0.6)
    s1, s2 = 1.7 * np.sin(0.2 + 0.3), 1.7 * np.sin(1.2 + 0.3)
    assert np.allclose(r1[0] * s2, r2[0] * s1, rtol=1e-12, atol=1e-14)
    assert np.abs(r1[1:]).max() == 0.0
    assert np.abs(r1[0]).max() > 0.1


@pytest.mark.slow
def test_manufactured_solution_rates():
    """Paper Section 6.1 (observed rates): the pressure error against the manufactured solution
    with c^2 = 1 + sin sin sin / 2 projected to P^M falls like h^r, r = min(N+1, M+3) (N=2,
    M=1: r = 3) and r = 2 for M = 0 (N=2, M=0)."""
    from workloads import c2_sinusoid, manufactured_solution, manufactured_source
    T = 0.2
    for M, want in ((1, 3.0), (0, 2.0)):
        errs = []
        for n in (2, 4):
            xyz, etov = kuhn_cube_mesh(n)
            o = Oracle(xyz, etov, 2, M)
            o.set_c2_function(c2_sinusoid, project=True)
            o.set_source(manufactured_source(c2_sinusoid), omega=np.pi)
            fns = [lambda x, y, z, i=i: manufactured_solution(x, y, z, 0.0)[i] for i in range(4)]
            Q = o.project_initial(fns)
            nsteps = 8 * n
            Q, _ = o.step(Q, np.zeros_like(Q), T / nsteps, nsteps)
            ex = [lambda x, y, z, i=i: manufactured_solution(x, y, z, T)[i] for i in range(4)]
            errs.append(np.sqrt(o.l2_error_sq(Q, ex)[0]))
        rate = np.log2(errs[0] / errs[1])
        assert rate > want - 0.6, (M, errs, rate)
