"""Polynomial bases on the reference tetrahedron, written from their definitions.

Test infrastructure only (see the package docstring).

* ``dubiner_tet``: the orthonormal (PKDO / Dubiner) basis in collapsed coordinates,
  with exact first derivatives from forward-mode automatic differentiation of the
  Jacobi three-term recurrence.
* ``bernstein_tet``: B^N_alpha = N!/(alpha!) lambda^alpha with the barycentric
  coordinates of paper Section 2: lambda_0 = -(1+r+s+t)/2, lambda_1 = (1+r)/2,
  lambda_2 = (1+s)/2, lambda_3 = (1+t)/2.

Coefficient order of Bernstein arrays (an interface format, shared with the library's
documentation): alpha = (a0, a1, a2, a3), |alpha| = N, graded by s = a1 + a2 + a3
(0..N); within one s, a3 ascending (outer) then a2 ascending (inner); a1 = s - a2 - a3,
a0 = N - s. Face arrays: (b0, b1, b2) graded by t = b1 + b2, then b2 ascending.
"""
from __future__ import annotations

from math import factorial, gamma, sqrt

import numpy as np


# ---------------------------------------------------------------- dual numbers
class Dual:
    """Value plus gradient with respect to (r, s, t), elementwise over arrays."""

    __slots__ = ("v", "g")

    def __init__(self, v, g):
        self.v = np.asarray(v, dtype=np.float64)
        self.g = np.asarray(g, dtype=np.float64)

    @staticmethod
    def const(c, shape):
        return Dual(np.full(shape, float(c)), np.zeros((3,) + tuple(shape)))

    def __add__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v + o.v, self.g + o.g)
        return Dual(self.v + o, self.g)

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.v, -self.g)

    def __sub__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v - o.v, self.g - o.g)
        return Dual(self.v - o, self.g)

    def __rsub__(self, o):
        return Dual(o - self.v, -self.g)

    def __mul__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v * o.v, self.g * o.v + self.v * o.g)
        return Dual(self.v * o, self.g * o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v / o.v, (self.g * o.v - self.v * o.g) / (o.v * o.v))
        return Dual(self.v / o, self.g / o)

    def __rtruediv__(self, o):
        return Dual(o / self.v, -o * self.g / (self.v * self.v))

    def ipow(self, n: int):
        out = Dual(np.ones_like(self.v), np.zeros_like(self.g))
        for _ in range(n):
            out = out * self
        return out


# -------------------------------------------------------------- Jacobi polynomials
def _jacobi_norm_sq(n: int, a: float, b: float) -> float:
    """Integral of (1-x)^a (1+x)^b P_n^{(a,b)}(x)^2 over [-1, 1] (standard normalisation)."""
    return (2.0 ** (a + b + 1.0) / (2 * n + a + b + 1.0)
            * gamma(n + a + 1.0) * gamma(n + b + 1.0) / (gamma(n + a + b + 1.0) * factorial(n)))


def jacobi_orthonormal(x, nmax: int, a: float, b: float):
    """Orthonormal Jacobi polynomials P_0..P_nmax at x (x may be a ``Dual``).

    Standard three-term recurrence for P_n^{(a,b)}, then division by sqrt of the norm.
    """
    out = []
    one = x * 0.0 + 1.0
    p0 = one
    out.append(p0)
    if nmax >= 1:
        p1 = ((a + b + 2.0) * x + (a - b)) * 0.5
        out.append(p1)
    for n in range(2, nmax + 1):
        s = 2 * n + a + b
        c1 = 2.0 * n * (n + a + b) * (s - 2.0)
        c2 = (s - 1.0) * (s * (s - 2.0))
        c3 = (s - 1.0) * (a * a - b * b)
        c4 = 2.0 * (n + a - 1.0) * (n + b - 1.0) * s
        pn = ((c2 * x + c3) * out[n - 1] - c4 * out[n - 2]) / c1
        out.append(pn)
    return [out[n] * (1.0 / sqrt(_jacobi_norm_sq(n, a, b))) for n in range(nmax + 1)]


# --------------------------------------------------------------- orthonormal basis
def dubiner_indices(N: int):
    """(i, j, k) with i + j + k <= N, ordered by total degree then lexicographically."""
    idx = []
    for d in range(N + 1):
        for i in range(d + 1):
            for j in range(d - i + 1):
                idx.append((i, j, d - i - j))
    return idx


def dubiner_tet(N: int, r, s, t, grad: bool = False):
    """Orthonormal Dubiner basis of P^N on the reference tetrahedron at points (r, s, t).

    psi_ijk = 2 sqrt(2) P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i P_k^{(2i+2j+2,0)}(c) (1-c)^{i+j}
    with collapsed coordinates a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t.
    Points must not lie on the collapsed edge or vertex (quadrature points never do).

    Returns V [npts, Np] (and, with ``grad``, a list [Vr, Vs, Vt]).
    """
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    shape = r.shape
    z = np.zeros(shape)
    o = np.ones(shape)
    R = Dual(r, np.stack([o, z, z]))
    S = Dual(s, np.stack([z, o, z]))
    T = Dual(t, np.stack([z, z, o]))
    if np.any(np.abs(s + t) < 1e-14) or np.any(np.abs(1.0 - t) < 1e-14):
        raise ValueError("point on a collapsed edge of the Dubiner map")
    a = 2.0 * (1.0 + R) / (-1.0 * S - T) - 1.0
    b = 2.0 * (1.0 + S) / (1.0 - T) - 1.0
    c = T
    cols = []
    pa = jacobi_orthonormal(a, N, 0.0, 0.0)
    for (i, j, k) in dubiner_indices(N):
        pb = jacobi_orthonormal(b, j, 2.0 * i + 1.0, 0.0)[j]
        pc = jacobi_orthonormal(c, k, 2.0 * (i + j) + 2.0, 0.0)[k]
        f = 2.0 * sqrt(2.0) * pa[i] * pb * (1.0 - b).ipow(i) * pc * (1.0 - c).ipow(i + j)
        cols.append(f)
    V = np.stack([f.v for f in cols], axis=-1)
    if not grad:
        return V
    G = [np.stack([f.g[d] for f in cols], axis=-1) for d in range(3)]
    return V, G


# ----------------------------------------------------------------- Bernstein basis
def multi_indices(N: int):
    """Multi-indices (a0, a1, a2, a3), |alpha| = N, in the documented coefficient order."""
    out = []
    for s in range(N + 1):
        for a3 in range(s + 1):
            for a2 in range(s - a3 + 1):
                out.append((N - s, s - a2 - a3, a2, a3))
    return out


def multi_indices_2d(N: int):
    """Face multi-indices (b0, b1, b2), |beta| = N, in the documented order."""
    out = []
    for t in range(N + 1):
        for b2 in range(t + 1):
            out.append((N - t, t - b2, b2))
    return out


def barycentric(r, s, t):
    """lambda_0..3 of the reference tetrahedron (paper Section 2)."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return np.stack([-(1.0 + r + s + t) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0, (1.0 + t) / 2.0])


def bernstein_tet(N: int, r, s, t):
    """Matrix [npts, Np] of B^N_alpha(r, s, t) = N!/alpha! prod_j lambda_j^alpha_j."""
    lam = barycentric(np.atleast_1d(r), np.atleast_1d(s), np.atleast_1d(t))
    cols = []
    for al in multi_indices(N):
        coef = factorial(N) / np.prod([factorial(a) for a in al])
        col = coef * np.ones(lam.shape[1])
        for j in range(4):
            col = col * lam[j] ** al[j]
        cols.append(col)
    return np.stack(cols, axis=-1)


def bernstein_tri(N: int, mu):
    """Matrix [npts, Nfp] of 2D Bernstein polynomials at barycentric points mu [3, npts]."""
    cols = []
    for be in multi_indices_2d(N):
        coef = factorial(N) / np.prod([factorial(b) for b in be])
        col = coef * np.ones(mu.shape[1])
        for j in range(3):
            col = col * mu[j] ** be[j]
        cols.append(col)
    return np.stack(cols, axis=-1)


def bernstein_eval(N: int, coef, r, s, t):
    """Evaluate Bernstein coefficient arrays [..., Np] at reference points -> [..., npts]."""
    B = bernstein_tet(N, r, s, t)
    return np.asarray(coef) @ B.T
