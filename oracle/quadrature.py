"""Gauss-Jacobi rules and collapsed (Duffy/Stroud) rules on the reference simplices.

Test infrastructure only (see the package docstring).

The paper uses Xiao-Gimbutas rules of degree 2N+1 for N <= 7 and a collapsed-coordinate
rule for N > 7 (Section 6.3.2). The oracle uses collapsed Gauss-Jacobi rules for all N:
with n points per direction they integrate polynomials of total degree 2n-1 exactly,
which is all that the weight-adjusted operators need once c^2 is a polynomial.
"""
from __future__ import annotations

from math import gamma

import numpy as np


def gauss_jacobi(n: int, alpha: float, beta: float):
    """n-point Gauss rule for the weight (1-x)^alpha (1+x)^beta on [-1, 1].

    Golub-Welsch: the nodes are the eigenvalues of the symmetric Jacobi matrix of the
    three-term recurrence of the monic Jacobi polynomials, the weights are mu0 times the
    squared first components of the normalised eigenvectors.
    """
    if n < 1:
        raise ValueError("n >= 1")
    a, b = float(alpha), float(beta)
    diag = np.empty(n)
    for i in range(n):
        s = 2 * i + a + b
        if i == 0:
            diag[i] = (b - a) / (a + b + 2.0)
        else:
            diag[i] = (b * b - a * a) / (s * (s + 2.0))
    off = np.empty(max(n - 1, 0))
    for i in range(1, n):
        s = 2 * i + a + b
        num = 4.0 * i * (i + a) * (i + b) * (i + a + b)
        den = s * s * (s + 1.0) * (s - 1.0)
        off[i - 1] = np.sqrt(num / den)
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(T)
    mu0 = 2.0 ** (a + b + 1.0) * gamma(a + 1.0) * gamma(b + 1.0) / gamma(a + b + 2.0)
    w = mu0 * V[0, :] ** 2
    return x, w


def tri_rule(n: int):
    """Collapsed rule on the reference triangle {r, s >= -1, r + s <= 0} (area 2).

    (a, b) in [-1,1]^2 maps to r = (1+a)(1-b)/2 - 1, s = b, with Jacobian (1-b)/2.
    Exact for total degree 2n-1. Returns (r, s, w).
    """
    xa, wa = gauss_jacobi(n, 0.0, 0.0)
    xb, wb = gauss_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    r = (1.0 + A) * (1.0 - B) / 2.0 - 1.0
    s = B
    w = WA * WB / 2.0
    return r.ravel(), s.ravel(), w.ravel()


def tet_rule(n: int):
    """Collapsed rule on the reference tetrahedron {r,s,t >= -1, r+s+t <= -1} (volume 4/3).

    (a, b, c) in [-1,1]^3 maps to r = (1+a)(1-b)(1-c)/4 - 1, s = (1+b)(1-c)/2 - 1, t = c,
    with Jacobian (1-b)(1-c)^2/8; the (1-b) and (1-c)^2 factors are absorbed into
    Gauss-Jacobi weights. Exact for total degree 2n-1. Returns (r, s, t, w).
    """
    xa, wa = gauss_jacobi(n, 0.0, 0.0)
    xb, wb = gauss_jacobi(n, 1.0, 0.0)
    xc, wc = gauss_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    r = (1.0 + A) * (1.0 - B) * (1.0 - C) / 4.0 - 1.0
    s = (1.0 + B) * (1.0 - C) / 2.0 - 1.0
    t = C
    w = WA * WB * WC / 8.0
    return r.ravel(), s.ravel(), t.ravel(), w.ravel()


def points_for_degree(deg: int) -> int:
    """Points per direction for a collapsed rule exact to total degree ``deg``."""
    return max(1, (deg + 2) // 2)
