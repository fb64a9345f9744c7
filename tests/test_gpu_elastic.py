"""The elastic weight-adjusted update on the device (Bernstein products and telescoped
projections) against the quadrature oracle, on the same seeded Bernstein inputs."""
import numpy as np
import pytest

from oracle import Oracle
from oracle.elastic import elastic_update
from workloads import c2_gaussian_bumps, c2_sinusoid, kuhn_cube_mesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1808_08645_amd as bb
    bb.load_library()
    return bb


def _media(K, Mp, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.5, 1.5, (K, Mp)), rng.uniform(0.5, 2.0, (K, Mp)), rng.uniform(0.3, 1.0, (K, Mp)))


def _compare(o, out_gpu, ref_modal):
    a = o.bernstein_values_at_quad(out_gpu.double().cpu().numpy())
    b = o.values_at_quad(ref_modal)
    return o.rel_l2(a, b)


CASES = [(1, 0), (1, 1), (2, 2), (3, 1), (4, 2), (5, 1), (5, 2), (6, 3), (7, 2), (8, 4), (9, 4)]


@pytest.mark.parametrize("N,M", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_elastic_update_matches_oracle(bb, N, M, dtype):
    print(f"[elastic] N={N} M={M} {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(2)
    etov = etov[:37]  # a ragged element count
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    K, Np, Mp = s.K, s.Np, s.Mp
    r = np.random.default_rng(90 + N).standard_normal((9, K, Np))
    rho_inv, lam, mu = _media(K, Mp, 91 + M)
    if dtype == "f32":
        r, rho_inv, lam, mu = (x.astype(np.float32).astype(np.float64) for x in (r, rho_inv, lam, mu))
    s.elastic_set_media(rho_inv, lam, mu)
    import torch
    rd = torch.as_tensor(r, device="cuda").to(torch.float64 if dtype == "f64" else torch.float32).contiguous()
    out = s.elastic_update(rd)
    o = Oracle(xyz, etov, N, M)
    ref = elastic_update(o, o.from_bernstein(r), rho_inv, lam, mu)
    err = _compare(o, out, ref)
    tol = 1e-11 if dtype == "f64" else 1e-5
    assert np.all(err < tol), err


def test_elastic_full_size_sampled(bb):
    """196,608 tets, N=5, M=2, media projected from smooth fields; the oracle checks 300
    sampled elements (the update is local to an element)."""
    import torch
    print("[elastic full size]", flush=True)
    xyz, etov = kuhn_cube_mesh(32)
    s = bb.Solver(xyz, etov, 5, 2)
    rho_inv, lam, mu = s.elastic_set_media(lambda x, y, z: 1.0 / (1.0 + 0.3 * x), c2_gaussian_bumps(0),
                                           lambda x, y, z: 0.5 * c2_sinusoid(x, y, z))
    r = np.random.default_rng(95).standard_normal((9, s.K, s.Np))
    out = s.elastic_update(torch.as_tensor(r, device="cuda").contiguous()).cpu().numpy()
    sel = np.sort(np.random.default_rng(96).choice(s.K, 300, replace=False))
    o = Oracle(xyz, etov[sel], 5, 2)
    ref = elastic_update(o, o.from_bernstein(r[:, sel]), rho_inv[sel], lam[sel], mu[sel])
    err = o.rel_l2(o.bernstein_values_at_quad(out[:, sel]), o.values_at_quad(ref))
    assert np.all(err < 1e-11), err


def test_elastic_error_paths(bb):
    import torch
    print("[elastic errors]", flush=True)
    xyz, etov = kuhn_cube_mesh(1)
    s = bb.Solver(xyz, etov, 2, 1)
    r = torch.zeros((9, s.K, s.Np), dtype=torch.float64, device="cuda")
    with pytest.raises(bb.BBWADGError) as ei:
        s.elastic_update(r)
    assert ei.value.code == -3
    bad = np.ones((s.K, s.Mp))
    bad[0, 0] = np.inf
    with pytest.raises(bb.BBWADGError) as ei:
        s.elastic_set_media(bad, np.ones_like(bad), np.ones_like(bad))
    assert ei.value.code == -3
    with pytest.raises(ValueError):
        s.elastic_update(torch.zeros((4, s.K, s.Np), dtype=torch.float64, device="cuda"))
    # valid media, then media that are not positive: the weights 1/rho, mu and 3 lambda + 2 mu
    # must be positive everywhere; a rejected call leaves the previous media in place
    one = np.ones((s.K, s.Mp))
    s.elastic_set_media(one, one, one)
    rr = torch.as_tensor(np.random.default_rng(5).standard_normal((9, s.K, s.Np)), device="cuda")
    before = s.elastic_update(rr).cpu()
    for rho_inv, lam, mu in [(-one, one, one), (one, one, -0.5 * one), (one, -one, one)]:
        with pytest.raises(bb.BBWADGError) as ei:
            s.elastic_set_media(rho_inv, lam, mu)
        assert ei.value.code == -3
    assert torch.equal(s.elastic_update(rr).cpu(), before)
    s.set_c2_policy(True)  # the accepting policy stores them
    s.elastic_set_media(one, -one, one)


@pytest.mark.parametrize("N,M", [(1, 0), (2, 1), (3, 3), (5, 2), (7, 3), (9, 4)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_wadg_update_matches_oracle(bb, N, M, dtype):
    """The acoustic update on its own, Pi_N(c^2_M r), against P_q diag(c^2_M) V_q r."""
    import torch
    from workloads import random_c2_coefficients
    print(f"[wadg update] N={N} M={M} {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(2)
    etov = etov[:29]
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    c2 = random_c2_coefficients(97, s.K, s.Mp)
    r = np.random.default_rng(98).standard_normal((s.K, s.Np))
    if dtype == "f32":
        c2, r = c2.astype(np.float32).astype(np.float64), r.astype(np.float32).astype(np.float64)
    s.set_c2(c2)
    out = s.wadg_update(torch.as_tensor(r, device="cuda").to(torch.float64 if dtype == "f64" else torch.float32))
    o = Oracle(xyz, etov, N, M)
    o.set_c2_bernstein(c2)
    Rm = o.from_bernstein(r[None])[0]
    ref = ((Rm @ o.Vq.T) * o.c2q) @ o.Pq.T
    err = o.rel_l2(o.bernstein_values_at_quad(out.double().cpu().numpy()[None]), o.values_at_quad(ref[None]))
    tol = 1e-11 if dtype == "f64" else 1e-5
    assert np.all(err < tol), err


def test_wadg_update_full_size_equals_dense_update(bb):
    """196,608 tets, N=5, M=2: the Bernstein update and the dense quadrature update with c^2_M at
    the points compute the same projection."""
    import torch
    print("[wadg update full size]", flush=True)
    xyz, etov = kuhn_cube_mesh(32)
    s = bb.Solver(xyz, etov, 5, 2)
    s.project_c2(c2_gaussian_bumps(0))
    s.dense_set_c2(None)
    r = torch.as_tensor(np.random.default_rng(99).standard_normal((s.K, s.Np)), device="cuda")
    a = s.wadg_update(r)
    b = s.dense_update(r)
    rel = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    assert rel < 1e-12, rel
