"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds only input data: mesh vertex coordinates and element-to-vertex
lists, material fields c^2(x), initial-condition functions and seeded random
arrays. It contains none of the method's arithmetic (no geometry factors, no
connectivity, no basis, no projection); each side derives those itself.

Workloads (all on the unit cube [0,1]^3, split into n^3 hexahedra and each hexahedron
into the 6 Kuhn tetrahedra that share its main diagonal, so the mesh is conforming):

* ``cube_sinusoid``  -- the paper's 3D test medium c^2 = 1 + 0.5 sin(pi x) sin(pi y) sin(pi z)
  (Section 6.1) with the standing-wave-like start p = cos(pi x)cos(pi y)cos(pi z), u = 0.
* ``cube_bumps``     -- c^2 = 1 + sum of 8 seeded Gaussian bumps (amplitude U[-0.4,0.4],
  width 0.1), Gaussian pressure pulse of width 0.05 at the cube centre.
* ``cube_layers``    -- three-layer medium c^2 in {1, 2, 4} split by two parallel planes with
  a seeded tilted normal, so the interfaces cut through elements (sub-cell jumps).

The paper's own meshes (GMSH, a 7,854-element timing mesh) are not available; these
structured Kuhn meshes stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "kuhn_cube_mesh",
    "c2_sinusoid",
    "c2_gaussian_bumps",
    "c2_three_layer",
    "ic_cos_product",
    "ic_gaussian_pulse",
    "exact_sin_mode",
    "exact_cos_mode",
    "manufactured_solution",
    "manufactured_source",
    "receiver_grid",
    "c2_random_model",
    "grid_centres",
    "random_state",
    "random_c2_coefficients",
    "dim_p",
    "CONFIGS",
]

# The six permutations of the axes; each gives one Kuhn tetrahedron
# v000 -> v000+e_a -> v000+e_a+e_b -> v111 inside a unit cell.
_KUHN_PATHS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def dim_p(n: int) -> int:
    """Dimension of the degree-n polynomial space on a tetrahedron, (n+1)(n+2)(n+3)/6."""
    return (n + 1) * (n + 2) * (n + 3) // 6


def kuhn_cube_mesh(n: int, order: str = "tiled", tile: int = 4):
    """Unit cube split into n^3 cells x 6 Kuhn tetrahedra.

    Returns ``(xyz, etov)``: ``xyz`` float64 [Nv, 3], ``etov`` int32 [6 n^3, 4].
    Each row of ``etov`` lists its vertex ids in ascending order (the Kuhn split is
    conforming, so every interior face is shared by exactly two tetrahedra).

    ``order`` sets the element order: ``"lex"`` numbers cells x-fastest; ``"tiled"``
    numbers cells in tile^3 blocks (blocks x-fastest, cells x-fastest inside a block)
    so that face neighbours sit close together in memory.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    # vertex id = i + (n+1) * (j + (n+1) * k)
    ids = np.arange((n + 1) ** 3)
    i = ids % (n + 1)
    j = (ids // (n + 1)) % (n + 1)
    k = ids // (n + 1) ** 2
    xyz = np.stack([i / n, j / n, k / n], axis=1).astype(np.float64)

    def vid(a, b, c):
        return a + (n + 1) * (b + (n + 1) * c)

    cells = []
    if order == "lex":
        for c in range(n):
            for b in range(n):
                for a in range(n):
                    cells.append((a, b, c))
    elif order == "tiled":
        t = max(1, int(tile))
        nb = (n + t - 1) // t
        for C in range(nb):
            for B in range(nb):
                for A in range(nb):
                    for c in range(C * t, min(n, (C + 1) * t)):
                        for b in range(B * t, min(n, (B + 1) * t)):
                            for a in range(A * t, min(n, (A + 1) * t)):
                                cells.append((a, b, c))
    else:
        raise ValueError("order must be 'lex' or 'tiled'")
    cells = np.asarray(cells, dtype=np.int64)
    etov = np.empty((6 * len(cells), 4), dtype=np.int64)
    for p, path in enumerate(_KUHN_PATHS):
        corner = cells.copy()
        v = [vid(corner[:, 0], corner[:, 1], corner[:, 2])]
        for ax in path:
            corner[:, ax] += 1
            v.append(vid(corner[:, 0], corner[:, 1], corner[:, 2]))
        etov[p::6] = np.stack(v, axis=1)
    etov.sort(axis=1)
    return xyz, etov.astype(np.int32)


# --------------------------------------------------------------------------- media
def c2_sinusoid(x, y, z):
    """c^2 = 1 + 0.5 sin(pi x) sin(pi y) sin(pi z) (the paper's 3D medium, Section 6.1)."""
    return 1.0 + 0.5 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def _bump_params(seed: int):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(-0.4, 0.4, size=8)
    ctr = rng.uniform(0.0, 1.0, size=(8, 3))
    return amp, ctr


def c2_gaussian_bumps(seed: int = 0, width: float = 0.1):
    """c^2 = 1 + sum_i A_i exp(-|x - x_i|^2 / (2 w^2)), A_i ~ U[-0.4, 0.4], x_i ~ U[0,1]^3.

    Returns a vectorised callable f(x, y, z). The parameters are drawn from
    ``numpy.random.default_rng(seed)``; with 8 bumps of |A| <= 0.4 the field stays
    above 1 - 8*0.4 only in the worst overlap, so callers check positivity.
    """
    amp, ctr = _bump_params(seed)

    def f(x, y, z):
        x = np.asarray(x, dtype=np.float64)
        out = np.ones(np.broadcast(x, y, z).shape)
        for a, c in zip(amp, ctr):
            r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
            out = out + a * np.exp(-r2 / (2.0 * width * width))
        return out

    f.params = (amp, ctr, width)
    return f


def c2_three_layer(seed: int = 1, values=(1.0, 2.0, 4.0)):
    """Three-layer medium split by two parallel planes n.x = s1, s2.

    n = normalize(a, b, 1) with a, b ~ U[-0.25, 0.25] from ``default_rng(seed)``;
    s1, s2 split [min n.x, max n.x] over the unit cube into thirds. The layers take
    c^2 = values[0], values[1], values[2] from low to high n.x.
    """
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(-0.25, 0.25, size=2)
    nrm = np.array([a, b, 1.0])
    nrm /= np.linalg.norm(nrm)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float)
    d = corners @ nrm
    lo, hi = d.min(), d.max()
    s1 = lo + (hi - lo) / 3.0
    s2 = lo + 2.0 * (hi - lo) / 3.0

    def f(x, y, z):
        t = nrm[0] * np.asarray(x) + nrm[1] * np.asarray(y) + nrm[2] * np.asarray(z)
        return np.where(t < s1, values[0], np.where(t < s2, values[1], values[2])).astype(np.float64)

    f.params = (nrm, s1, s2, values)
    return f


# ----------------------------------------------------------------- initial states
def ic_cos_product(x, y, z):
    """p = cos(pi x) cos(pi y) cos(pi z)."""
    return np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z)


def ic_gaussian_pulse(x, y, z, centre=(0.5, 0.5, 0.5), width=0.05):
    """p = exp(-|x - centre|^2 / (2 width^2))."""
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return np.exp(-r2 / (2.0 * width * width))


def exact_sin_mode(x, y, z, t):
    """Exact c = 1 solution for p = 0 walls: returns (p, u, v, w).

    p = sin(pi x) sin(pi y) sin(pi z) cos(w t), u = -(1/sqrt 3)(cos sin sin, ...) sin(w t),
    with w = sqrt(3) pi.
    """
    w = np.sqrt(3.0) * np.pi
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx, cy, cz = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    s = np.sin(w * t) / np.sqrt(3.0)
    return (sx * sy * sz * np.cos(w * t), -cx * sy * sz * s, -sx * cy * sz * s, -sx * sy * cz * s)


def manufactured_solution(x, y, z, t):
    """The 3D manufactured solution of paper Section 6.1: returns (p, u, v, w) with
    p = sin(pi x) sin(pi y) sin(pi z) cos(pi t) and u = -(cos sin sin, sin cos sin,
    sin sin cos) sin(pi t); p = 0 on the walls of the unit cube."""
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx, cy, cz = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    st = np.sin(np.pi * t)
    return (sx * sy * sz * np.cos(np.pi * t), -cx * sy * sz * st, -sx * cy * sz * st, -sx * sy * cz * st)


def manufactured_source(c2):
    """Spatial part g of the source f = g(x) sin(pi t) that makes manufactured_solution solve
    (1/c^2) p_t + div u = f, u_t + grad p = 0: g = (3 - 1/c^2) pi sin(pi x) sin(pi y) sin(pi z)."""
    def g(x, y, z):
        return (3.0 - 1.0 / c2(x, y, z)) * np.pi * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    return g


def _random_model_params(seed: int):
    rng = np.random.default_rng(10_000 + int(seed))
    a, b = rng.uniform(-0.3, 0.3, size=2)
    nrm = np.array([a, b, 1.0])
    nrm /= np.linalg.norm(nrm)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float) @ nrm
    nl = int(rng.integers(2, 5))
    cuts = np.sort(rng.uniform(corners.min(), corners.max(), size=nl - 1))
    vals = rng.uniform(1.0, 3.5, size=nl)
    amp = rng.uniform(-0.5, 0.5, size=4)
    wid = rng.uniform(0.08, 0.2, size=4)
    ctr = rng.uniform(0.0, 1.0, size=(4, 3))
    return nrm, cuts, vals, amp, wid, ctr


def c2_random_model(seed: int, transition: float = 0.03):
    """A seeded velocity model with c^2 in [1, 4]: 2-4 layers split by parallel planes with a
    tilted normal (a, b, 1)/|.|, a, b ~ U[-0.3, 0.3], interface offsets ~ U over the cube's
    extent along the normal, layer values ~ U[1, 3.5], each interface a tanh step of the given
    width (0.03 keeps the degree-2 projection on the 16^3 Kuhn mesh positive: sharp jumps of
    this size make it negative in about one medium in five); plus 4 Gaussian bumps (amplitude
    U[-0.5, 0.5], width U[0.08, 0.2], centres U[0, 1]^3); clipped to [1, 4]."""
    nrm, cuts, vals, amp, wid, ctr = _random_model_params(seed)

    def f(x, y, z):
        x, y, z = np.broadcast_arrays(np.asarray(x, dtype=np.float64), y, z)
        d = nrm[0] * x + nrm[1] * y + nrm[2] * z
        out = vals[0] + np.zeros_like(d)
        for i, ct in enumerate(cuts):
            out = out + (vals[i + 1] - vals[i]) * 0.5 * (1.0 + np.tanh((d - ct) / transition))
        for A, w, c in zip(amp, wid, ctr):
            out = out + A * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2.0 * w * w))
        return np.clip(out, 1.0, 4.0)

    return f


def c2_random_model_family(seed: int, transition: float = 0.03):
    """The medium of c2_random_model(seed) before its clipping, written as a linear combination
    c^2(x) = sum_i theta_i phi_i(x): phi_i are the smooth indicators of the layers (differences
    of the tanh steps) and the 4 Gaussian bumps, theta = (layer values, bump amplitudes).
    Returns (phis, theta) with theta the model's own parameters."""
    nrm, cuts, vals, amp, wid, ctr = _random_model_params(seed)

    def step(i):
        def h(x, y, z):
            x, y, z = np.broadcast_arrays(np.asarray(x, dtype=np.float64), y, z)
            d = nrm[0] * x + nrm[1] * y + nrm[2] * z
            return 0.5 * (1.0 + np.tanh((d - cuts[i]) / transition))
        return h

    H = [step(i) for i in range(len(cuts))]
    phis = []
    for j in range(len(vals)):
        def layer(x, y, z, j=j):
            lo = H[j - 1](x, y, z) if j > 0 else 1.0
            hi = H[j](x, y, z) if j < len(H) else 0.0
            return np.broadcast_to(np.asarray(lo - hi, dtype=np.float64), np.broadcast(x, y, z).shape)
        phis.append(layer)
    for w, c in zip(wid, ctr):
        def bump(x, y, z, w=w, c=c):
            x, y, z = np.broadcast_arrays(np.asarray(x, dtype=np.float64), y, z)
            return np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2.0 * w * w))
        phis.append(bump)
    return phis, np.concatenate([vals, amp])


def grid_centres(n: int = 16):
    """Cell centres ((i + 1/2)/n) of an n^3 grid on the unit cube as (x, y, z) arrays of shape
    [n, n, n] indexed [z, y, x]."""
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return x, y, z


def receiver_grid(n: int = 8, z: float = 1.0, shift=(0.5, 0.53125)):
    """n x n receiver points ((i + sx)/n, (j + sy)/n, z) on a plane z = const, row-major in
    (j, i). The default shift keeps them off the cell edges and face diagonals of the Kuhn
    meshes with 8m cells per side, so each lies in the interior of one boundary face."""
    i, j = np.meshgrid(np.arange(n), np.arange(n))
    x = (i.ravel() + shift[0]) / n
    y = (j.ravel() + shift[1]) / n
    return np.stack([x, y, np.full(n * n, float(z))], axis=1)


def exact_cos_mode(x, y, z, t):
    """Exact c = 1 solution for rigid walls (u.n = 0): returns (p, u, v, w).

    p = cos(pi x) cos(pi y) cos(pi z) cos(w t), u = (1/sqrt 3)(sin cos cos, ...) sin(w t).
    """
    w = np.sqrt(3.0) * np.pi
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx, cy, cz = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    s = np.sin(w * t) / np.sqrt(3.0)
    return (cx * cy * cz * np.cos(w * t), sx * cy * cz * s, cx * sy * cz * s, cx * cy * sz * s)


# ------------------------------------------------------------------ random arrays
def random_state(seed: int, K: int, Np: int, dtype=np.float64):
    """Seeded coefficient array of shape [4, K, Np], entries U[-1, 1]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(4, K, Np)).astype(dtype)


def random_c2_coefficients(seed: int, K: int, Mp: int, lo: float = 0.5, hi: float = 2.0):
    """Seeded per-element coefficient array [K, Mp] with entries U[lo, hi] (all positive)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(K, Mp)).astype(np.float64)


# ------------------------------------------------------------------ named configs
CONFIGS = {
    # 4x4x4 cells x 6 = 384 tets, N=3, M=1, sinusoidal medium, 10 LSRK4 steps at CFL 0.5
    "cube384_N3_M1": dict(cells=4, N=3, M=1, medium="sinusoid", ic="cos", bc="p0",
                          steps=10, cfl=0.5, dtype="f64"),
    # 32x32x32 cells x 6 = 196,608 tets, N=5, M=2, Gaussian-bump medium, pulse, 200 steps
    "cube196k_N5_M2": dict(cells=32, N=5, M=2, medium="bumps", ic="pulse", bc="p0",
                           steps=200, cfl=0.5, dtype="f64"),
    # same mesh, N=4..9, M=N//2, three-layer medium, FP32 vs FP64
    "cube196k_layers": dict(cells=32, N=(4, 5, 6, 7, 8, 9), M="N//2", medium="layers",
                            ic="pulse", bc="p0", steps=200, cfl=0.5, dtype=("f32", "f64")),
}
