"""Host side of the library on the CPU: exported symbols, geometry and connectivity,
FP64 projections (the c^2 setup step), c_j tables and error handling.

Contexts here are created in host-only mode, which makes no HIP call, so these tests run
without a GPU. Geometry and projections are compared with the oracle's own independent
code; the c_j table with the paper's printed values.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import Oracle
from oracle.mesh import Mesh
from workloads import (c2_gaussian_bumps, c2_sinusoid, c2_three_layer, ic_cos_product, ic_gaussian_pulse,
                       kuhn_cube_mesh)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bb():
    from tests._build import ensure_built
    ensure_built()
    import paper_1808_08645_amd as bb
    return bb


def test_library_exports_every_declared_symbol(bb):
    inc = os.path.join(ROOT, "include")
    header = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    declared = set(re.findall(r"^\s*(?:int|int32_t|int64_t|const char\*)\s+(bbwadg_\w+)\s*\(", header, re.M))
    assert declared, "no declarations parsed"
    lib = C.CDLL(bb.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(bb.EXPORTS)


def test_geometry_and_connectivity_match_oracle_mesh(bb):
    xyz, etov = kuhn_cube_mesh(3)
    rng = np.random.default_rng(0)
    etov_shuffled = np.array([rng.permutation(r) for r in etov], dtype=np.int32)
    s = bb.Solver(xyz, etov_shuffled, 3, 1, host_only=True)
    ev = s.element_vertices()
    assert np.array_equal(ev, np.sort(etov_shuffled, axis=1))
    g = s.geometry()
    m = Mesh(xyz, ev)
    assert np.allclose(g["J"], m.J, rtol=1e-14)
    assert np.allclose(g["G"], m.G, atol=1e-12)
    assert np.allclose(g["normal"], m.normal, atol=1e-14)
    assert np.allclose(g["Fscale"], m.Fscale, rtol=1e-13)
    nbr = g["nbr"]
    assert np.array_equal(nbr < 0, m.nbr < 0)
    inter = nbr >= 0
    assert np.array_equal((nbr >> 2)[inter], m.nbr[inter])
    assert np.array_equal((nbr & 3)[inter], m.nbr_face[inter])


@pytest.mark.parametrize("deg,fn", [(1, c2_sinusoid), (2, c2_gaussian_bumps(0)), (3, ic_cos_product),
                                    (5, ic_gaussian_pulse), (2, c2_three_layer(1)), (9, ic_cos_product)])
def test_projection_matches_oracle_projection(bb, deg, fn):
    """FP64 L^2 projection onto P^deg (same collapsed rule, independent code): compared as
    functions at the oracle's quadrature points."""
    xyz, etov = kuhn_cube_mesh(2)
    s = bb.Solver(xyz, etov, max(deg, 1), 0, host_only=True)
    coef = s.project_function(fn, deg)
    o = Oracle(xyz, etov, deg, 0)
    from oracle.basis import bernstein_tet, dubiner_tet
    modal = o.project_modal(fn, deg)
    V = dubiner_tet(deg, o.rq, o.sq, o.tq)
    B = bernstein_tet(deg, o.rq, o.sq, o.tq)
    a, b = coef @ B.T, modal @ V.T
    rel = np.sqrt(o.l2_sq((a - b)[None]) / o.l2_sq(b[None]))[0]
    assert rel < 1e-12, rel


def test_c2_callback_equals_sample_projection(bb):
    xyz, etov = kuhn_cube_mesh(2)
    s = bb.Solver(xyz, etov, 3, 2, host_only=True)
    ref = s.project_function(c2_sinusoid, 2)
    s.project_c2_callback(lambda x, y, z: float(c2_sinusoid(x, y, z)))
    assert np.allclose(s.get_c2(), ref, rtol=0, atol=1e-15)


def _read_golden(name):
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        if line.strip() and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


def test_library_cj_tables_match_paper(bb):
    for row in _read_golden("tab1_projection_cj.txt"):
        N, M = int(row[0]), int(row[1])
        assert np.allclose(bb.projection_coefficients(N, M), row[2:], atol=5.1e-5)
    for row in _read_golden("tab2_massinv_cj.txt"):
        N = int(row[0])
        assert np.allclose(bb.projection_coefficients(N, -1), row[1:], rtol=1e-13)
    for N, M, val, rtol in _read_golden("cond_sums.txt"):
        s = np.abs(bb.projection_coefficients(int(N), int(M))).sum()
        assert abs(s - val) <= rtol * val


def test_suggest_dt_formula(bb):
    xyz, etov = kuhn_cube_mesh(4)
    s = bb.Solver(xyz, etov, 3, 1, host_only=True)
    with pytest.raises(bb.BBWADGError):
        s.suggest_dt(0.5)  # c^2 not set yet
    coef = s.project_c2(c2_sinusoid)
    dt = s.suggest_dt(0.5)
    fs = s.geometry()["Fscale"].max()
    assert np.isclose(dt, 0.5 / (np.sqrt(coef.max()) * (4 * 6 / 3) * fs))


def test_error_paths(bb):
    xyz, etov = kuhn_cube_mesh(1)
    E = bb.BBWADGError
    for N, M in [(0, 0), (10, 0), (3, 4), (6, 5), (2, -1)]:
        with pytest.raises(E) as ei:
            bb.Solver(xyz, etov, N, M, host_only=True)
        assert ei.value.code == -1
    with pytest.raises(E):
        bb.Solver(xyz, etov, 3, 1, tau_p=-1.0, host_only=True)
    bad = etov.copy()
    bad[0, 0] = len(xyz) + 5
    with pytest.raises(E) as ei:
        bb.Solver(xyz, bad, 3, 1, host_only=True)
    assert ei.value.code == -1
    # degenerate: four coplanar vertices
    flat_xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    with pytest.raises(E) as ei:
        bb.Solver(flat_xyz, np.array([[0, 1, 2, 3]], np.int32), 2, 1, host_only=True)
    assert ei.value.code == -2
    # a face shared by three elements
    x3 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1]], float)
    with pytest.raises(E) as ei:
        bb.Solver(x3, np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], np.int32), 2, 1, host_only=True)
    assert ei.value.code == -2
    # c^2 checks
    s = bb.Solver(xyz, etov, 3, 1, host_only=True)
    c = np.ones((s.K, s.Mp))
    c[2, 1] = -5.0
    with pytest.raises(E) as ei:
        s.set_c2(c)
    assert ei.value.code == -3
    c[2, 1] = np.nan
    with pytest.raises(E) as ei:
        s.set_c2(c)
    assert ei.value.code == -3
    with pytest.raises(E) as ei:
        s.get_c2()
    assert ei.value.code == -3
    # hot path on a host-only context is refused
    lib = bb.load_library()
    assert lib.bbwadg_rhs(s._ctx, None, None, 0.0, None) == -1
    assert lib.bbwadg_step(s._ctx, None, None, 0.0, 0.1, 1, None) == -1
    assert b"host-only" in lib.bbwadg_last_error()
    out = (C.c_double * 4)()
    assert lib.bbwadg_energy(s._ctx, None, 0, s.K, out, None) == -1
    assert lib.bbwadg_l2error2(s._ctx, None, 0, s.K, None, out, None) == -1
    assert lib.bbwadg_project_fn(s._ctx, bb.bbwadg.C2_CALLBACK(lambda x, y, z, u: 0.0), None, 0, None, None) == -1
    assert b"host-only" in lib.bbwadg_last_error()
    for bad in [(-1, 0, 0), (0, -2, 1), (5, 5, 4)]:
        assert lib.bbwadg_coef_index(*bad) == -1


def test_coef_index_matches_documented_order(bb):
    """bbwadg_coef_index against the oracle's enumeration of the multi-indices."""
    from oracle.basis import multi_indices
    for N in (1, 4, 9, 13):
        for i, (a0, a1, a2, a3) in enumerate(multi_indices(N)):
            assert bb.coef_index(a1, a2, a3) == i


def test_dense_rule_points_match_oracle_volume_rule(bb):
    """The dense WADG rule is the oracle's volume rule (exact to degree 2N+M): same points."""
    xyz, etov = kuhn_cube_mesh(1)
    for N, M in [(2, 1), (5, 2), (9, 4)]:
        s = bb.Solver(xyz, etov, N, M, host_only=True)
        o = Oracle(xyz, etov, N, M)
        n = (2 * N + M + 2) // 2
        assert s.dense_npoints() == n ** 3 == len(o.wq)
        X = s.dense_points()
        Y = o.mesh.map_points(o.rq, o.sq, o.tq)
        for k in range(s.K):
            a = X[k][np.lexsort(X[k].T)]
            b = Y[k][np.lexsort(Y[k].T)]
            assert np.allclose(a, b, atol=1e-13)


def test_receiver_location_matches_oracle(bb):
    """The library and the oracle place receivers in the same elements (lowest-numbered
    containing element), including points on shared faces and on the boundary."""
    from oracle.adjoint import locate
    from workloads import receiver_grid
    xyz, etov = kuhn_cube_mesh(4)
    s = bb.Solver(xyz, etov, 3, 1, host_only=True)
    pts = np.concatenate([receiver_grid(8, 1.0), receiver_grid(4, 0.5, shift=(0.0, 0.0)),
                          np.random.default_rng(8).uniform(0, 1, (30, 3))])
    s.set_receivers(pts)
    o = Oracle(xyz, etov, 3, 1)
    elem, _ = locate(o.mesh, pts)
    assert np.array_equal(s.receiver_elements(), elem)
    with pytest.raises(bb.BBWADGError):
        s.set_receivers([[0.5, 0.5, 1.2]])
    with pytest.raises(bb.BBWADGError):
        s.set_receivers([[0.5, np.nan, 0.2]])
