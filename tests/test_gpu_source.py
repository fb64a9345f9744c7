"""The pressure source of the manufactured-solution study (paper Section 6.1) on the device.

* parity of the right-hand side and of LSRK4 steps with a source against the CPU oracle
  (each side projects c^2 and the source with its own code, or both take the same seeded
  Bernstein coefficients);
* the observed convergence rates of the paper's 3D manufactured solution,
  r = min(N+1, M+3) for M >= 1 and r = 2 for M = 0, with c^2 = 1 + sin sin sin / 2
  projected onto P^M.
"""
import numpy as np
import pytest

from oracle import Oracle
from workloads import (c2_sinusoid, kuhn_cube_mesh, manufactured_solution, manufactured_source,
                       random_c2_coefficients, random_state)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11


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


def _fields(t):
    return [lambda x, y, z, i=i: manufactured_solution(x, y, z, t)[i] for i in range(4)]


@pytest.mark.parametrize("N,M", [(1, 0), (2, 1), (5, 2), (9, 4)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rhs_with_source_parity(bb, N, M, dtype):
    """Random state, c^2 and source coefficients; time factor 0.8 sin(2.5 t + 0.4) at t = 0.31."""
    print(f"[rhs source] N={N} M={M} {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(2)
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    q = random_state(51, s.K, s.Np)
    c2 = random_c2_coefficients(52, s.K, s.Mp)
    g = random_state(53, s.K, s.Np)[0]
    if dtype == "f32":  # both sides take the single-precision source
        g = g.astype(np.float32).astype(np.float64)
    s.set_c2(c2)
    s.set_source(g, amp=0.8, omega=2.5, phase=0.4)
    out = s.rhs(s.to_device(q), t=0.31)
    o = Oracle(xyz, etov, N, M)
    o.set_c2_bernstein(c2)
    o.set_source(o.from_bernstein(g[None])[0], amp=0.8, omega=2.5, phase=0.4)
    err = _compare(o, out, o.rhs(o.from_bernstein(q), t=0.31))
    tol = FP64_TOL if dtype == "f64" else 1e-5
    assert np.all(err < tol), err
    # removing the source gives the source-free right-hand side back
    s.set_source(None)
    o.src = None
    err = _compare(o, s.rhs(s.to_device(q), t=0.31), o.rhs(o.from_bernstein(q)))
    assert np.all(err < tol), err


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_step_with_source_parity(bb, dtype):
    """384 tets, N=3, M=1: the manufactured problem from t0 = 0.05 for 12 steps; the stage
    times t0 + (n + c_k) dt enter through the source."""
    import torch
    print(f"[step source] {dtype}", flush=True)
    xyz, etov = kuhn_cube_mesh(4)
    N, M = 3, 1
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    o = Oracle(xyz, etov, N, M)
    s.project_c2(c2_sinusoid)
    o.set_c2_function(c2_sinusoid, project=True)
    g = manufactured_source(c2_sinusoid)
    s.set_source(g, omega=np.pi)
    o.set_source(g, omega=np.pi)
    t0, dt, n = 0.05, 0.004, 12
    q = s.to_device(s.initial_state(_fields(t0)))
    res = torch.zeros_like(q)
    s.step(q, res, dt, n, t0=t0)
    torch.cuda.synchronize()
    Q, _ = o.step(o.project_initial(_fields(t0)), np.zeros((4, s.K, s.Np)), dt, n, t0=t0)
    err = _compare(o, q, Q)
    tol = FP64_TOL if dtype == "f64" else 1e-5
    assert np.all(err < tol), err


def _manufactured_error(bb, n, N, M, T, cfl=0.5):
    """Per-field squared L^2 errors (p, u, v, w) of the manufactured problem at time T."""
    import torch
    xyz, etov = kuhn_cube_mesh(n)
    s = bb.Solver(xyz, etov, N, M)
    s.project_c2(c2_sinusoid)
    s.set_source(manufactured_source(c2_sinusoid), omega=np.pi)
    nsteps = int(np.ceil(T / s.suggest_dt(cfl)))
    q = s.to_device(s.initial_state(_fields(0.0)))
    res = torch.zeros_like(q)
    s.step(q, res, T / nsteps, nsteps)
    torch.cuda.synchronize()
    return s.l2error2(q, _fields(T))


@pytest.mark.parametrize("N,M", [(2, 1), (3, 1), (4, 0), (4, 1), (4, 2)])
def test_manufactured_solution_convergence_rates(bb, N, M):
    """Paper Section 6.1 (the 3D convergence study, plotted there for N = 4 and 5): the L^2 error
    of the pressure at T = 0.5 on the 4^3, 8^3 and 16^3 Kuhn cubes falls at the rate
    r = 2 for M = 0, else min(N+1, M+3): the rate between the two finest meshes is within 0.3
    of r. (The velocity error falls one order slower for M >= 1, at M + 2 when that is below
    N + 1; it is printed, not checked.)"""
    r = 2 if M == 0 else min(N + 1, M + 3)
    E = np.array([_manufactured_error(bb, n, N, M, 0.5) for n in (4, 8, 16)])
    ep, eu = np.sqrt(E[:, 0]), np.sqrt(E[:, 1:].sum(1))
    rp, ru = np.log2(ep[:-1] / ep[1:]), np.log2(eu[:-1] / eu[1:])
    print(f"[rates] N={N} M={M} p errors {ep} rates {rp} (expected {r}); u rates {ru}", flush=True)
    assert abs(rp[-1] - r) < 0.3, (ep, rp)


def test_dense_rhs_with_source_matches_oracle_wadg(bb):
    """The quadrature WADG right-hand side with the true c^2 and a source: the oracle's plain
    WADG with the same source."""
    print("[dense source]", flush=True)
    xyz, etov = kuhn_cube_mesh(2)
    N, M = 4, 1
    s = bb.Solver(xyz, etov, N, M)
    s.dense_set_c2(c2_sinusoid)
    g = random_state(54, s.K, s.Np)[0]
    s.set_source(g, amp=1.3, omega=0.7, phase=-0.2)
    q = s.to_device(random_state(55, s.K, s.Np))
    out = s.rhs_dense(q, t=0.9)
    o = Oracle(xyz, etov, N, M)
    o.set_c2_function(c2_sinusoid, project=False)
    o.set_source(o.from_bernstein(g[None])[0], amp=1.3, omega=0.7, phase=-0.2)
    err = _compare(o, out, o.rhs(o.from_bernstein(q.cpu().numpy()), t=0.9))
    assert np.all(err < FP64_TOL), err


def test_source_error_paths(bb):
    print("[source errors]", flush=True)
    xyz, etov = kuhn_cube_mesh(1)
    s = bb.Solver(xyz, etov, 2, 1)
    g = np.ones((s.K, s.Np))
    g[1, 3] = np.nan
    with pytest.raises(bb.BBWADGError) as ei:
        s.set_source(g)
    assert ei.value.code == -1
    with pytest.raises(bb.BBWADGError):
        s.set_source(np.ones((s.K, s.Np)), omega=np.inf)
    with pytest.raises(ValueError):
        s.set_source(np.ones((s.K, s.Np + 1)))


def test_full_size_rhs_with_source_on_sampled_elements(bb):
    """196,608 tets, N=5, M=2 (the benchmark's launch configuration) with the manufactured
    source at t = 0.3: the oracle recomputes 200 sampled elements with their face neighbours."""
    print("[full-size source]", flush=True)
    xyz, etov = kuhn_cube_mesh(32)
    s = bb.Solver(xyz, etov, 5, 2)
    s.project_c2(c2_sinusoid)
    g = manufactured_source(c2_sinusoid)
    s.set_source(g, amp=1.2, omega=np.pi)
    q = random_state(71, s.K, s.Np)
    out = s.rhs(s.to_device(q), t=0.3).cpu().numpy()
    rng = np.random.default_rng(72)
    seeds = np.unique(np.concatenate([rng.choice(s.K, 196, replace=False), [0, s.K - 1]]))
    nbr = s.geometry()["nbr"]
    sub = set(int(k) for k in seeds)
    for k in seeds:
        sub.update(int(v) >> 2 for v in nbr[k] if v >= 0)
    sub = np.array(sorted(sub))
    o = Oracle(xyz, etov[sub], 5, 2)
    o.set_c2_function(c2_sinusoid, project=True)
    o.set_source(g, amp=1.2, omega=np.pi)
    R = o.rhs(o.from_bernstein(q[:, sub]), t=0.3)
    pos = np.searchsorted(sub, seeds)
    a = o.bernstein_values_at_quad(out[:, seeds])
    b = o.values_at_quad(R[:, pos])
    wJ = o.mesh.J[pos][:, None] * o.wq[None, :]
    err = np.sqrt(np.sum((a - b) ** 2 * wJ, axis=(1, 2)) / np.sum(b ** 2 * wJ, axis=(1, 2)))
    assert np.all(err < FP64_TOL), err.max()
