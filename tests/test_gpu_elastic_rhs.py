"""The elastic DG right-hand side on the device (Bernstein derivative and elevation stencils,
fluxes on face coefficients, Bernstein lift, then the weight-adjusted update) against the
quadrature oracle, on the same seeded Bernstein states, on a jittered ragged mesh with both
wall conditions."""
import numpy as np
import pytest

from oracle import Oracle
from oracle.elastic import elastic_rhs
from workloads import kuhn_cube_mesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1808_08645_amd as bb
    bb.load_library()
    return bb


def _mesh(n, keep, seed):
    xyz, etov = kuhn_cube_mesh(n)
    assert np.all(np.diff(etov, axis=1) > 0)  # vertices ascending: same local order on both sides
    xyz = xyz + np.random.default_rng(seed).uniform(-0.06 / n, 0.06 / n, xyz.shape)
    return xyz, etov[:keep]


def _media(K, Mp, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.5, 1.5, (K, Mp)), rng.uniform(0.5, 2.0, (K, Mp)), rng.uniform(0.3, 1.0, (K, Mp)))


CASES = [(1, 0), (2, 1), (3, 2), (4, 2), (5, 2), (6, 3), (7, 2), (8, 4), (9, 4)]


@pytest.mark.parametrize("N,M", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("wall", ["free", "rigid"])
def test_elastic_rhs_matches_oracle(bb, N, M, dtype, wall):
    import torch
    print(f"[elastic rhs] N={N} M={M} {dtype} {wall}", flush=True)
    xyz, etov = _mesh(2, 37, 7)
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    K, Np, Mp = s.K, s.Np, s.Mp
    q = np.random.default_rng(120 + N).standard_normal((9, K, Np))
    media = _media(K, Mp, 121 + M)
    if dtype == "f32":
        q = q.astype(np.float32).astype(np.float64)
        media = tuple(x.astype(np.float32).astype(np.float64) for x in media)
    s.elastic_set_media(*media)
    td = torch.float64 if dtype == "f64" else torch.float32
    qd = torch.as_tensor(q, device="cuda").to(td).contiguous()
    tau_v, tau_s = 0.7, 1.3
    o = Oracle(xyz, etov, N, M)
    qm = o.from_bernstein(q)
    tol = 1e-10 if dtype == "f64" else (2e-5 if N <= 6 else 3e-4)
    for weighted in (False, True):
        out = s.elastic_rhs(qd, wall=wall, tau_v=tau_v, tau_s=tau_s, weighted=weighted)
        torch.cuda.synchronize()
        ref = elastic_rhs(o, qm, media if weighted else None, tau_v=tau_v, tau_s=tau_s, wall=wall)
        err = o.rel_l2(o.bernstein_values_at_quad(out.double().cpu().numpy()), o.values_at_quad(ref))
        assert np.all(err < tol), (weighted, err)


def test_elastic_rhs_full_size_sampled(bb):
    """196,608 tets, N=5, M=2, traction-free walls: the oracle recomputes 40 sampled elements
    with their neighbours' states (the right-hand side of an element reads only its face
    neighbours)."""
    import torch
    print("[elastic rhs full size]", flush=True)
    xyz, etov = kuhn_cube_mesh(32)
    s = bb.Solver(xyz, etov, 5, 2)
    q = np.random.default_rng(130).standard_normal((9, s.K, s.Np))
    out = s.elastic_rhs(torch.as_tensor(q, device="cuda").contiguous(), weighted=False).cpu().numpy()
    rng = np.random.default_rng(131)
    sel = np.sort(rng.choice(s.K, 40, replace=False))
    has = lambda v: (etov == v).any(axis=1)
    errs = []
    for k in sel:
        # element k with its face neighbours: a sub-mesh in which k's faces are interior exactly
        # where they are interior in the full mesh
        ids = [int(k)]
        for f in range(4):
            a, b, c = (int(etov[k, v]) for v in range(4) if v != f)
            nb = np.nonzero(has(a) & has(b) & has(c))[0]
            ids += [int(x) for x in nb if x != k]
        ids = np.array(ids)
        o = Oracle(xyz, etov[ids], 5, 2)
        ref = elastic_rhs(o, o.from_bernstein(q[:, ids]), None, wall="free")
        a = o.bernstein_values_at_quad(out[:, ids[:1]])
        b = o.values_at_quad(ref)[:, :1]
        errs.append(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))
    assert max(errs) < 1e-11, max(errs)


def test_elastic_rhs_errors(bb):
    import torch
    print("[elastic rhs errors]", flush=True)
    xyz, etov = kuhn_cube_mesh(1)
    s = bb.Solver(xyz, etov, 3, 1)
    q = torch.zeros((9, s.K, s.Np), dtype=torch.float64, device="cuda")
    with pytest.raises(bb.BBWADGError, match="media"):
        s.elastic_rhs(q, weighted=True)
    with pytest.raises(bb.BBWADGError, match="tau"):
        s.elastic_rhs(q, tau_v=-1.0, weighted=False)
    with pytest.raises(ValueError):
        s.elastic_rhs(q, wall="absorbing")
    with pytest.raises(ValueError):
        s.elastic_rhs(q[:4])
    assert torch.count_nonzero(s.elastic_rhs(q, weighted=False)) == 0


@pytest.mark.parametrize("N,M", [(1, 0), (3, 2), (5, 2), (7, 3), (9, 4)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_elastic_step_matches_oracle(bb, N, M, dtype):
    """Three low-storage RK4 steps of the weighted elastic system (rigid walls) against the
    oracle's, from a smooth state projected in FP64."""
    import torch
    from oracle.elastic import elastic_step
    print(f"[elastic step] N={N} M={M} {dtype}", flush=True)
    xyz, etov = _mesh(2, 37, 8)
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    K, Np, Mp = s.K, s.Np, s.Mp
    media = _media(K, Mp, 140 + M)
    q = np.random.default_rng(141 + N).standard_normal((9, K, Np)) / N
    if dtype == "f32":
        q = q.astype(np.float32).astype(np.float64)
        media = tuple(x.astype(np.float32).astype(np.float64) for x in media)
    s.elastic_set_media(*media)
    dt = 0.02 / (N + 1) ** 2
    td = torch.float64 if dtype == "f64" else torch.float32
    qd = torch.as_tensor(q, device="cuda").to(td).contiguous()
    rd = torch.zeros_like(qd)
    s.elastic_step(qd, rd, dt, 3, wall="rigid")
    torch.cuda.synchronize()
    o = Oracle(xyz, etov, N, M)
    qm, _ = elastic_step(o, o.from_bernstein(q), np.zeros((9, K, Np)), dt, 3, media, wall="rigid")
    err = o.rel_l2(o.bernstein_values_at_quad(qd.double().cpu().numpy()), o.values_at_quad(qm))
    tol = 1e-11 if dtype == "f64" else (2e-6 if N <= 6 else 2e-5)
    assert np.all(err < tol), err


def _energy(o, qb, rho_inv, lam, mu):
    """1/2 int rho |v|^2 + sigma : C^{-1} sigma over the mesh for media constant per element
    (Voigt shear components are engineering strains: sigma_s = mu gamma_s)."""
    V = o.bernstein_values_at_quad(qb)  # [9, K, nq]
    wJ = o.mesh.J[:, None] * o.wq[None, :]
    rho = 1.0 / rho_inv[:, :1]
    kin = rho * np.sum(V[:3] ** 2, axis=0)
    lam, mu = lam[:, :1], mu[:, :1]
    tr = V[3] + V[4] + V[5]
    normal = (np.sum(V[3:6] ** 2, axis=0) - lam / (3.0 * lam + 2.0 * mu) * tr ** 2) / (2.0 * mu)
    shear = np.sum(V[6:9] ** 2, axis=0) / mu
    return 0.5 * float(np.sum(wJ * (kin + normal + shear)))


@pytest.mark.parametrize("N", [3, 5])
@pytest.mark.parametrize("wall", ["free", "rigid"])
def test_elastic_step_energy_never_grows(bb, N, wall):
    """Media constant per element (M = 0, where the weight-adjusted mass is the exact weighted
    mass): the discrete energy of the device time steps is non-increasing, and the penalty
    fluxes make it decrease (energy stability of the scheme, any mesh size)."""
    import torch
    print(f"[elastic energy] N={N} {wall}", flush=True)
    xyz, etov = _mesh(2, 48, 9)
    s = bb.Solver(xyz, etov, N, 0)
    rng = np.random.default_rng(150 + N)
    K = s.K
    rho_inv, lam, mu = rng.uniform(0.5, 1.5, (K, 1)), rng.uniform(0.5, 2.0, (K, 1)), rng.uniform(0.3, 1.0, (K, 1))
    s.elastic_set_media(rho_inv, lam, mu)
    o = Oracle(xyz, etov, N, 0)
    q = torch.as_tensor(rng.standard_normal((9, K, s.Np)), device="cuda").contiguous()
    res = torch.zeros_like(q)
    dt = 0.02 / (N + 1) ** 2
    e = [_energy(o, q.cpu().numpy(), rho_inv, lam, mu)]
    for _ in range(8):
        s.elastic_step(q, res, dt, 5, wall=wall)
        e.append(_energy(o, q.cpu().numpy(), rho_inv, lam, mu))
    e = np.array(e)
    assert np.all(np.diff(e) <= 1e-12 * e[0]), e
    assert e[-1] < 0.999 * e[0] and e[-1] > 0.05 * e[0], e
