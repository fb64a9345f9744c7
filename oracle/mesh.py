"""Affine tetrahedral mesh geometry and face connectivity for the oracle.

Test infrastructure only (see the package docstring).

Element k is the image of the reference tetrahedron under x = sum_j lambda_j v_j, where
v_0..v_3 are its vertices in the order ``etov[k]`` gives them (paper Section 2), so
dx/dr = (v1 - v0)/2, dx/ds = (v2 - v0)/2, dx/dt = (v3 - v0)/2. Face f is the face
opposite local vertex f (lambda_f = 0). Matrix form (paper Section 3.1, eq. matform):
J is the volume Jacobian determinant, G_ij = d r_j / d x_i, and a face integral is
J_f times the integral over a reference triangle of area 2, so J_f = |face| / 2.
"""
from __future__ import annotations

import numpy as np


class Mesh:
    """Geometry and connectivity derived from vertex coordinates and ``etov``."""

    def __init__(self, xyz, etov):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.etov = np.asarray(etov, dtype=np.int64)
        K = self.etov.shape[0]
        self.K = K
        V = self.xyz[self.etov]  # [K, 4, 3]
        self.verts = V
        A = np.stack([(V[:, 1] - V[:, 0]) / 2.0, (V[:, 2] - V[:, 0]) / 2.0,
                      (V[:, 3] - V[:, 0]) / 2.0], axis=2)  # A[k, i, j] = d x_i / d r_j
        self.A = A
        detA = np.linalg.det(A)
        if np.any(np.abs(detA) < 1e-300):
            raise ValueError("degenerate element")
        self.J = np.abs(detA)  # |det|; orientation only flips the sign
        Ainv = np.linalg.inv(A)  # Ainv[k, j, i] = d r_j / d x_i
        self.G = np.transpose(Ainv, (0, 2, 1))  # G[k, i, j] = d r_j / d x_i
        # faces: face f is opposite local vertex f; its vertices in increasing local order
        self.face_local = [tuple(v for v in range(4) if v != f) for f in range(4)]
        nrm = np.zeros((K, 4, 3))
        area = np.zeros((K, 4))
        for f in range(4):
            a, b, c = self.face_local[f]
            e1 = V[:, b] - V[:, a]
            e2 = V[:, c] - V[:, a]
            cr = np.cross(e1, e2)
            ar = 0.5 * np.linalg.norm(cr, axis=1)
            n = cr / (2.0 * ar)[:, None]
            # outward: away from the opposite vertex
            sgn = np.sign(np.einsum("ki,ki->k", n, V[:, a] - V[:, f]))
            nrm[:, f] = n * sgn[:, None]
            area[:, f] = ar
        self.normal = nrm
        self.area = area
        self.Jf = area / 2.0
        self.Fscale = self.Jf / self.J[:, None]
        self._connect()

    def _connect(self):
        """Neighbour element and face of each face, matched by the sorted global vertex triple."""
        K = self.K
        table = {}
        nbr = -np.ones((K, 4), dtype=np.int64)
        nbr_face = -np.ones((K, 4), dtype=np.int64)
        for k in range(K):
            for f in range(4):
                key = tuple(sorted(int(self.etov[k, v]) for v in self.face_local[f]))
                if key in table:
                    k2, f2 = table.pop(key)
                    nbr[k, f], nbr_face[k, f] = k2, f2
                    nbr[k2, f2], nbr_face[k2, f2] = k, f
                else:
                    table[key] = (k, f)
        self.nbr = nbr
        self.nbr_face = nbr_face
        # for interior faces: local positions, in the neighbour, of this face's three vertices
        pos = -np.ones((K, 4, 3), dtype=np.int64)
        for k in range(K):
            for f in range(4):
                k2 = nbr[k, f]
                if k2 < 0:
                    continue
                ids2 = list(self.etov[k2])
                for m, v in enumerate(self.face_local[f]):
                    pos[k, f, m] = ids2.index(int(self.etov[k, v]))
        self.nbr_pos = pos

    def map_points(self, r, s, t):
        """Physical coordinates [K, npts, 3] of reference points on every element."""
        lam = np.stack([-(1.0 + r + s + t) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0,
                        (1.0 + t) / 2.0])  # [4, npts]
        return np.einsum("jq,kjd->kqd", lam, self.verts)
