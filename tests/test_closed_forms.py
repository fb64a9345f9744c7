"""Closed forms behind the fast Bernstein operators, pinned against dense definitions.

The HIP path applies sparse Bernstein operators whose entries come from closed forms
(paper Sections 4 and 5). Here each closed form is written out in plain Python and
compared with what the definitions give: Bernstein polynomials evaluated from their
definition, dense mass matrices by exact quadrature, and the values the paper prints
(Tables 1 and 2, the conditioning sums of Section 5.4). No GPU and no HIP code.
"""
import os
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

from oracle.basis import bernstein_tet, bernstein_tri, multi_indices, multi_indices_2d
from oracle.quadrature import tet_rule, tri_rule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return rows


# ---- closed forms (as the kernels use them) --------------------------------------
def mass_eigenvalue(n, k):
    """Distinct eigenvalue k of the degree-n Bernstein mass matrix on the volume-4/3 tet:
    (4/3) 3! (n!)^2 / ((n-k)! (n+k+3)!)."""
    return Fraction(8 * factorial(n) ** 2, factorial(n - k) * factorial(n + k + 3))


def projection_cj(N, M, mass_inverse=False):
    """c_j of Theorem 5.3 (or of the mass-inverse representation): in the modal basis the
    elevation products are diagonal (Corollary A.3), which gives the triangular system
    sum_{j<=N-k} c_j lambda^{N-j}_k = lambda^{N+M}_k (or 1), k = N..0."""
    c = []
    for k in range(N, -1, -1):
        rhs = Fraction(1) if mass_inverse else mass_eigenvalue(N + M, k)
        s = sum(c[j] * mass_eigenvalue(N - j, k) for j in range(len(c)))
        c.append((rhs - s) / mass_eigenvalue(N - len(c), k))
    return c


def elevation(n, dim=3):
    """Dense one-degree elevation E^n_{n-1} [n_p x (n-1)_p] from eq. (bbele)."""
    mi = multi_indices if dim == 3 else multi_indices_2d
    A, B = mi(n), mi(n - 1)
    ib = {b: i for i, b in enumerate(B)}
    E = np.zeros((len(A), len(B)))
    for r, g in enumerate(A):
        for j in range(dim + 1):
            if g[j] > 0:
                gg = list(g)
                gg[j] -= 1
                E[r, ib[tuple(gg)]] += g[j] / n
    return E


def multiply(N, M, a, b):
    """eq. (mcoeff): c_gamma = sum_beta a_{gamma-beta} b_beta C(gamma,beta)/C(N+M,N)."""
    G, A, Bm = multi_indices(N + M), multi_indices(N), multi_indices(M)
    ia = {x: i for i, x in enumerate(A)}
    out = np.zeros(len(G))
    for r, g in enumerate(G):
        for jb, be in enumerate(Bm):
            d = tuple(x - y for x, y in zip(g, be))
            if min(d) < 0:
                continue
            w = np.prod([comb(g[i], be[i]) for i in range(4)]) / comb(N + M, N)
            out[r] += a[ia[d]] * b[jb] * w
    return out


def derivative_stencil(N, j, a):
    """(D^j a)_gamma = sum_{k: gamma_k>0} gamma_k a_{gamma - e_k + e_j}: the barycentric
    derivative d/d lambda_j, elevated back to degree N (at most 4 nonzeros per row)."""
    A = multi_indices(N)
    ia = {x: i for i, x in enumerate(A)}
    out = np.zeros(len(A))
    for r, g in enumerate(A):
        for k in range(4):
            if g[k] > 0:
                d = list(g)
                d[k] -= 1
                d[j] += 1
                out[r] += g[k] * a[ia[tuple(d)]]
    return out


def _rand_pts(n, seed=0):
    lam = np.random.default_rng(seed).dirichlet(np.ones(4), size=n).T
    return 2 * lam[1] - 1, 2 * lam[2] - 1, 2 * lam[3] - 1


# ---- tests -------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 2, 5, 9])
def test_derivative_stencil_is_exact(N):
    """(1/2)(D^1 - D^0) a are the degree-N Bernstein coefficients of d/dr of the polynomial."""
    a = np.random.default_rng(N).normal(size=len(multi_indices(N)))
    r, s, t = _rand_pts(7)
    h = 1e-5
    f = lambda r, s, t: bernstein_tet(N, r, s, t) @ a  # noqa: E731
    for j, (dr, ds, dt) in zip((1, 2, 3), [(h, 0, 0), (0, h, 0), (0, 0, h)]):
        fd = (f(r + dr, s + ds, t + dt) - f(r - dr, s - ds, t - dt)) / (2 * h)
        coef = 0.5 * (derivative_stencil(N, j, a) - derivative_stencil(N, 0, a))
        assert np.abs(bernstein_tet(N, r, s, t) @ coef - fd).max() < 1e-6 * max(1, np.abs(fd).max())
    # at most d+1 = 4 nonzeros per row
    eye = np.eye(len(a))
    for j in range(4):
        D = np.stack([derivative_stencil(N, j, eye[:, c]) for c in range(len(a))], axis=1)
        assert (np.count_nonzero(D, axis=1) <= 4).all()


@pytest.mark.parametrize("n", [1, 3, 8, 13])
def test_elevation_reproduces_polynomial(n):
    a = np.random.default_rng(n).normal(size=len(multi_indices(n - 1)))
    r, s, t = _rand_pts(9, n)
    E = elevation(n)
    assert np.abs(bernstein_tet(n, r, s, t) @ (E @ a) - bernstein_tet(n - 1, r, s, t) @ a).max() < 1e-13
    assert (np.count_nonzero(E, axis=1) <= 4).all()


@pytest.mark.parametrize("N,M", [(1, 1), (2, 1), (3, 2), (4, 2), (5, 2), (6, 3)])
def test_multiplication_identity(N, M):
    rng = np.random.default_rng(10 * N + M)
    a = rng.normal(size=len(multi_indices(N)))
    b = rng.normal(size=len(multi_indices(M)))
    c = multiply(N, M, a, b)
    r, s, t = _rand_pts(11, N)
    fg = (bernstein_tet(N, r, s, t) @ a) * (bernstein_tet(M, r, s, t) @ b)
    assert np.abs(bernstein_tet(N + M, r, s, t) @ c - fg).max() < 1e-12 * max(1, np.abs(fg).max())
    if M == 1:  # eq. (coeff): c_gamma = sum_j a_{gamma-e_j} b_j gamma_j/(N+1)
        G, A = multi_indices(N + 1), multi_indices(N)
        ia = {x: i for i, x in enumerate(A)}
        ej = [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)]
        bidx = [multi_indices(1).index(e) for e in ej]
        c1 = np.zeros(len(G))
        for rr, g in enumerate(G):
            for j in range(4):
                if g[j] > 0:
                    d = list(g)
                    d[j] -= 1
                    c1[rr] += a[ia[tuple(d)]] * b[bidx[j]] * g[j] / (N + 1)
        assert np.allclose(c1, c, atol=1e-14)


def test_cj_match_table1():
    for row in _read_rows("tab1_projection_cj.txt"):
        N, M = int(row[0]), int(row[1])
        c = [float(x) for x in projection_cj(N, M)]
        assert len(c) == len(row) - 2
        assert np.allclose(c, row[2:], atol=5.1e-5), (N, M, c)


def test_cj_match_table2_exactly():
    for row in _read_rows("tab2_massinv_cj.txt"):
        N = int(row[0])
        c = projection_cj(N, 0, mass_inverse=True)
        assert [float(x) for x in c] == row[1:]


def test_conditioning_sums():
    for N, M, val, rtol in _read_rows("cond_sums.txt"):
        c = projection_cj(int(N), 0, mass_inverse=True) if M < 0 else projection_cj(int(N), int(M))
        s = float(sum(abs(x) for x in c))
        assert abs(s - val) <= rtol * val, (N, M, s)


@pytest.mark.parametrize("N,M", [(1, 1), (2, 1), (3, 1), (3, 2), (4, 2), (5, 2), (6, 3)])
def test_telescoped_projection_equals_dense_l2_projection(N, M):
    """Theorem 5.3: sum_j c_j E^N_{N-j} (E^N_{N-j})^T (E^{N+M}_N)^T is the L^2 projection
    M_N^{-1} (E^{N+M}_N)^T M_{N+M} (mass matrices from exact quadrature)."""
    r, s, t, w = tet_rule(N + M + 1)
    BN = bernstein_tet(N, r, s, t)
    BH = bernstein_tet(N + M, r, s, t)
    dense = np.linalg.solve(BN.T @ (w[:, None] * BN), BN.T @ (w[:, None] * BH))
    c = [float(x) for x in projection_cj(N, M)]
    # E^N_{N-j}: chain of one-degree elevations; reduction is its transpose
    Ered = np.eye(len(multi_indices(N + M)))
    for n in range(N + M, N, -1):
        Ered = elevation(n).T @ Ered  # apply reductions degree n -> n-1
    P = np.zeros((len(multi_indices(N)), len(multi_indices(N))))
    Ej = np.eye(len(multi_indices(N)))
    for j in range(N + 1):
        P += c[j] * Ej @ Ej.T
        if j < N:
            Ej = Ej @ elevation(N - j)
    P = P @ Ered
    assert np.abs(P - dense).max() < 1e-9 * np.abs(dense).max()
    # reproduces P^N: the projection of an elevated degree-N polynomial is itself
    Eup = np.eye(len(multi_indices(N)))
    for n in range(N + 1, N + M + 1):
        Eup = elevation(n) @ Eup
    assert np.abs(P @ Eup - np.eye(len(multi_indices(N)))).max() < 1e-12
    # M = 0 gives c_0 = 1 and the identity
    assert float(projection_cj(N, 0)[0]) == 1.0 and all(x == 0 for x in projection_cj(N, 0)[1:])


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_lift_factorisation_equals_dense_lift(N):
    """L^f = M^{-1} M_f restricted to face f's columns equals the factorised form:
    layer i (alpha_f = i) holds l_i (E^T)^i L_0 g with L_0 = (2N+3)/2 I + N^2/2 E E^T (on
    the face) and l_i = (-1)^i C(N,i)/(i+1). Reference face of area 2."""
    r, s, t, w = tet_rule(N + 2)
    B = bernstein_tet(N, r, s, t)
    Mv = B.T @ (w[:, None] * B)
    r2, s2, wf = tri_rule(N + 2)
    mu = np.stack([-(r2 + s2) / 2, (1 + r2) / 2, (1 + s2) / 2])
    A, A2 = multi_indices(N), multi_indices_2d(N)
    for f in range(4):
        others = [v for v in range(4) if v != f]
        lam = np.zeros((4, len(wf)))
        for m, v in enumerate(others):
            lam[v] = mu[m]
        Bf = bernstein_tet(N, 2 * lam[1] - 1, 2 * lam[2] - 1, 2 * lam[3] - 1)
        Mf = Bf.T @ (wf[:, None] * Bf)
        i2 = {b: i for i, b in enumerate(A2)}
        fcols = [i for i, a in enumerate(A) if a[f] == 0]
        dense = np.zeros((len(A), len(A2)))
        Lfull = np.linalg.solve(Mv, Mf)
        for i in fcols:
            dense[:, i2[tuple(A[i][v] for v in others)]] = Lfull[:, i]
        E = elevation(N, dim=2)
        lev = [(2 * N + 3) / 2 * np.eye(len(A2)) + N * N / 2 * E @ E.T]
        assert (np.count_nonzero(np.abs(lev[0]) > 1e-14, axis=1) <= 7).all()
        for i in range(1, N + 1):
            lev.append(elevation(N - i + 1, dim=2).T @ lev[-1])
        fact = np.zeros_like(dense)
        for row, a in enumerate(A):
            i = a[f]
            ell = (-1) ** i * comb(N, i) / (i + 1)
            idx = multi_indices_2d(N - i).index(tuple(a[v] for v in others))
            fact[row] = ell * lev[i][idx]
        assert np.abs(fact - dense).max() < 1e-11 * np.abs(dense).max()
    # the 2D face Bernstein basis restricted from the volume one (geometric decomposition)
    Bt = bernstein_tri(N, mu)
    lam = np.zeros((4, len(wf)))
    lam[1:] = mu
    Bv = bernstein_tet(N, 2 * lam[1] - 1, 2 * lam[2] - 1, 2 * lam[3] - 1)
    for i, a in enumerate(A):
        if a[0] == 0:
            assert np.allclose(Bv[:, i], Bt[:, A2.index(a[1:])])
        else:
            assert np.abs(Bv[:, i]).max() < 1e-14
