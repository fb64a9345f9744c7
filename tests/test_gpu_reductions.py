"""Parity of the library's FP64 reductions (through the C ABI) with the CPU oracle: the
squared L^2 error against an exact solution, the acoustic energy terms, the squared L^2
norm, and the C-callback projection of a state field.

The reductions accumulate in FP64 in both dtypes; in FP32 the oracle takes the state and
c^2 rounded to single precision, so the FP64 tolerance (1e-11 relative) holds for both.
"""
import numpy as np
import pytest

from oracle import Oracle
from workloads import (c2_gaussian_bumps, exact_cos_mode, exact_sin_mode, ic_gaussian_pulse, kuhn_cube_mesh,
                       random_c2_coefficients, random_state)

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def bb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1808_08645_amd as bb
    bb.load_library()
    return bb


def dimp(n):
    return (n + 1) * (n + 2) * (n + 3) // 6


def _rounded(a, dtype):
    return a.astype(np.float32).astype(np.float64) if dtype == "f32" else a


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)


CASES = [(1, 0, 2), (3, 1, 2), (5, 2, 2), (6, 3, 1), (9, 4, 1)]


@pytest.mark.parametrize("N,M,n", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_energy_parity(bb, N, M, n, dtype):
    print(f"[energy] N={N} M={M} cube {n} {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(n)
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    q = random_state(41, s.K, s.Np)
    c2 = random_c2_coefficients(42, s.K, s.Mp)
    s.set_c2(c2)
    e = s.energy(s.to_device(q))
    o = Oracle(xyz, etov, N, M)
    o.set_c2_bernstein(_rounded(c2, dtype))
    ref = o.energy_terms(o.from_bernstein(_rounded(q, dtype)))
    assert np.all(_rel(e, ref) < TOL), (e, ref)


@pytest.mark.parametrize("N,M,n", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_l2error_parity(bb, N, M, n, dtype):
    print(f"[l2error] N={N} M={M} cube {n} {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(n)
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    q = random_state(43, s.K, s.Np) * 0.1
    fns = [lambda x, y, z, i=i: exact_sin_mode(x, y, z, 0.37)[i] for i in range(4)]
    err = s.l2error2(s.to_device(q), fns)
    o = Oracle(xyz, etov, N, M)
    ref = o.l2_error_sq(o.from_bernstein(_rounded(q, dtype)), fns)
    assert np.all(_rel(err, ref) < TOL), (err, ref)


def test_l2error_of_projected_solution_converges(bb):
    """Projected standing wave (rigid walls): error against it falls like h^{N+1}."""
    print("[l2error rate]", flush=True)
    errs = []
    N = 3
    for n in (2, 4):
        xyz, etov = kuhn_cube_mesh(n)
        s = bb.Solver(xyz, etov, N, 0, bc="rigid")
        fns = [lambda x, y, z, i=i: exact_cos_mode(x, y, z, 0.2)[i] for i in range(4)]
        q = s.to_device(s.initial_state(fns))
        errs.append(np.sqrt(s.l2error2(q, fns).sum()))
    assert np.log2(errs[0] / errs[1]) > N + 0.5, errs


def test_reduction_ranges_add_up_and_empty_range(bb):
    print("[ranges]", flush=True)
    xyz, etov = kuhn_cube_mesh(3)
    s = bb.Solver(xyz, etov, 4, 2)
    q = s.to_device(random_state(44, s.K, s.Np))
    s.set_c2(random_c2_coefficients(45, s.K, s.Mp))
    full = s.energy(q)
    parts = s.energy(q, 0, 37) + s.energy(q, 37, 101) + s.energy(q, 101, s.K)
    assert np.all(_rel(parts, full) < 1e-13)
    assert np.array_equal(s.energy(q, 50, 50), np.zeros(4))
    fns = [lambda x, y, z: np.cos(x + 2 * y) * z] * 4
    full = s.l2error2(q, fns)
    parts = s.l2error2(q, fns, 0, 64, chunk=17) + s.l2error2(q, fns, 64, s.K, chunk=50)
    assert np.all(_rel(parts, full) < 1e-13)
    with pytest.raises(bb.BBWADGError) as ei:
        s.energy(q, 5, s.K + 1)
    assert ei.value.code == -1


def test_l2norm_and_error_against_zero_agree(bb):
    """Two device routes to ||q||^2: closed-form mass matrix and the quadrature reduction."""
    import torch
    print("[norm routes]", flush=True)
    xyz, etov = kuhn_cube_mesh(3)
    s = bb.Solver(xyz, etov, 5, 2)
    q = s.to_device(random_state(46, s.K, s.Np))
    zero = torch.zeros((4, s.K, s.projection_npoints(5)), dtype=torch.float64, device="cuda")
    a = s.l2norm2(q)
    b = s.l2error2_samples(q, zero)
    assert np.all(_rel(a, b) < 1e-12), (a, b)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_energy_on_sampled_range(bb, dtype):
    """196,608 tets (N=5, M=2, bump medium, pulse): the energy of a ragged range of 1,003
    elements at the end of the mesh, against the oracle on those elements alone, and the
    energy of the whole mesh against the sum over the pieces."""
    print(f"[energy full size] {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(32)
    N, M = 5, 2
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    c2 = s.project_c2(c2_gaussian_bumps(0))
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    q0 = s.initial_state([ic_gaussian_pulse, lambda x, y, z: 0.1 * np.sin(3 * x), zero, zero])
    q = s.to_device(q0)
    k0, k1 = s.K - 1003, s.K
    e = s.energy(q, k0, k1)
    sub = s.element_vertices()[k0:k1]
    o = Oracle(xyz, sub, N, M)
    o.set_c2_bernstein(_rounded(c2[k0:k1], dtype))
    ref = o.energy_terms(o.from_bernstein(_rounded(q0[:, k0:k1], dtype)))
    assert np.all(_rel(e, ref) < TOL), (e, ref)
    full = s.energy(q)
    parts = sum(s.energy(q, a, min(s.K, a + 50000)) for a in range(0, s.K, 50000))
    assert np.all(_rel(parts, full) < 1e-12)
    assert full[0] > 0 and full[1] > 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_project_fn_callback_matches_oracle(bb, dtype):
    import torch
    print(f"[project_fn] {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(2)
    N = 4
    s = bb.Solver(xyz, etov, N, 1, dtype=dtype)
    q = s.empty_state()
    q.fill_(7.0)
    fn = lambda x, y, z: np.exp(-((x - 0.3) ** 2 + (y - 0.6) ** 2 + z * z))  # noqa: E731
    s.project_fn_callback(fn, 2, q)
    torch.cuda.synchronize()
    qc = q.double().cpu().numpy()
    assert np.all(qc[[0, 1, 3]] == 7.0)
    o = Oracle(xyz, etov, N, 1)
    ref = o.project_modal(fn, N)
    a = o.bernstein_values_at_quad(qc[2])
    b = o.values_at_quad(ref)
    rel = np.sqrt(o.l2_sq(a - b) / o.l2_sq(b))
    assert rel < (1e-12 if dtype == "f64" else 1e-6), rel
