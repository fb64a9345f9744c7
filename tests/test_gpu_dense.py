"""The dense quadrature WADG baseline (matrix-core kernel) through the C ABI.

* With c^2_M at the dense points it must equal the fast Bernstein right-hand side (the
  projection is exact for that rule: paper Theorem 5.3 against eq. pwadg).
* With the true c^2 at the points it must equal the oracle's plain WADG mode (c^2 point
  values at the same collapsed rule, dense quadrature matrices in an orthonormal basis).
Tolerance 1e-11 relative L2 per field (FP64); sizes span several 16-element tiles and a
ragged tail.
"""
import numpy as np
import pytest

from oracle import Oracle
from workloads import c2_gaussian_bumps, c2_sinusoid, kuhn_cube_mesh, random_c2_coefficients, random_state

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def bb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1808_08645_amd as bb
    bb.load_library()
    return bb


def _compare(o, q_gpu, Q_oracle):
    a = o.bernstein_values_at_quad(q_gpu.double().cpu().numpy())
    b = o.values_at_quad(Q_oracle)
    return o.rel_l2(a, b)


@pytest.mark.parametrize("N,M", [(1, 1), (2, 1), (3, 1), (4, 2), (5, 2), (6, 3), (7, 3), (8, 4), (9, 4)])
def test_dense_with_c2M_equals_bernstein_rhs(bb, N, M):
    print(f"[dense = bbwadg] N={N} M={M}", flush=True)
    xyz, etov = kuhn_cube_mesh(2)
    s = bb.Solver(xyz, etov, N, M)
    s.set_c2(random_c2_coefficients(61, s.K, s.Mp))
    q = s.to_device(random_state(62, s.K, s.Np))
    s.dense_set_c2(None)
    a = s.rhs(q)
    b = s.rhs_dense(q)
    o = Oracle(xyz, etov, N, M)
    o.set_c2_bernstein(s.get_c2())
    ref = o.rhs(o.from_bernstein(q.cpu().numpy()))
    assert np.all(_compare(o, a, ref) < TOL)
    assert np.all(_compare(o, b, ref) < TOL), _compare(o, b, ref)


@pytest.mark.parametrize("K_sel", [1, 7, 17, 48])
@pytest.mark.parametrize("N,M", [(3, 1), (5, 2)])
def test_dense_true_c2_matches_oracle_wadg(bb, K_sel, N, M):
    """Quadrature WADG of the true c^2 (the paper's comparison method)."""
    print(f"[dense true c2] K={K_sel} N={N} M={M}", flush=True)
    xyz, etov = kuhn_cube_mesh(2)
    etov = etov[:K_sel]
    s = bb.Solver(xyz, etov, N, M)
    s.dense_set_c2(c2_gaussian_bumps(3))
    q = s.to_device(random_state(63, s.K, s.Np))
    out = s.rhs_dense(q)
    o = Oracle(xyz, etov, N, M)
    o.set_c2_function(c2_gaussian_bumps(3), project=False)
    err = _compare(o, out, o.rhs(o.from_bernstein(q.cpu().numpy())))
    assert np.all(err < TOL), err


def test_dense_update_in_place_and_full_size_sample(bb):
    """196,608 tets, N=5, M=2: the update alone, in place and out of place, against the
    fast projection on a sample of elements (c^2_M at the points)."""
    import torch
    print("[dense full size]", flush=True)
    xyz, etov = kuhn_cube_mesh(32)
    s = bb.Solver(xyz, etov, 5, 2)
    s.project_c2(c2_sinusoid)
    s.dense_set_c2(None)
    q = s.to_device(random_state(64, s.K, s.Np))
    out = s.dense_update(q[0].contiguous())
    r = q[0].clone()
    s.dense_update(r, r)
    torch.cuda.synchronize()
    assert torch.equal(out, r)
    # the fast path computes the same projection: compare through the full right-hand sides
    a = s.rhs(q)
    b = s.rhs_dense(q)
    rel = torch.linalg.norm(a - b) / torch.linalg.norm(a)
    assert float(rel) < 1e-12, float(rel)


def test_dense_error_paths(bb):
    print("[dense errors]", flush=True)
    xyz, etov = kuhn_cube_mesh(1)
    s = bb.Solver(xyz, etov, 3, 1)
    q = s.empty_state()
    with pytest.raises(bb.BBWADGError) as ei:
        s.rhs_dense(q)
    assert ei.value.code == -3
    with pytest.raises(bb.BBWADGError) as ei:
        s.dense_set_c2(None)  # no c^2_M either
    assert ei.value.code == -3
    with pytest.raises(bb.BBWADGError) as ei:
        s.dense_set_c2(lambda x, y, z: 1.0 - 2.0 * x)  # not positive everywhere
    assert ei.value.code == -3
    s32 = bb.Solver(xyz, etov, 3, 1, dtype="f32")
    s32.set_c2(np.ones((s32.K, s32.Mp)))
    with pytest.raises(bb.BBWADGError) as ei:
        s32.dense_set_c2(None)
    assert ei.value.code == -1
