"""The receiver misfit and its gradient with respect to the c^2_M Bernstein coefficients on
the device, against the oracle's plain discrete adjoint (dense transposes, modal basis) and
against central finite differences of the device's own misfit.

Inputs: Kuhn-cube meshes, a Gaussian pressure pulse, seeded random c^2 coefficients and
seeded random observed traces (so that no expected value comes from the device).
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.adjoint import Receivers, misfit_gradient
from workloads import (c2_sinusoid, ic_gaussian_pulse, kuhn_cube_mesh, manufactured_source, random_c2_coefficients,
                       random_state, receiver_grid)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1808_08645_amd as bb
    bb.load_library()
    return bb


def _pulse(x, y, z):
    return ic_gaussian_pulse(x, y, z, centre=(0.4, 0.55, 0.5), width=0.2)


def _zero(x, y, z):
    return 0.0 * x


def _problem(bb, n, N, M, bc, dtype, seed):
    xyz, etov = kuhn_cube_mesh(n)
    s = bb.Solver(xyz, etov, N, M, dtype=dtype, bc=bc)
    c = random_c2_coefficients(seed, s.K, s.Mp)
    s.set_c2(c)
    q0 = s.initial_state([_pulse, _zero, _zero, _zero])
    return xyz, etov, s, c, q0


PTS = np.array([[0.3, 0.6, 1.0], [0.7, 0.2, 0.9], [0.5, 0.5, 0.5], [0.1, 0.8, 0.3], [0.9, 0.9, 0.05],
                [0.55, 0.45, 0.0]])


@pytest.mark.parametrize("n,N,M,bc,ckpt,dtype,source", [
    (2, 2, 1, "rigid", 3, "f64", False),
    (2, 3, 0, "p0", 2, "f64", True),
    (1, 4, 2, "rigid", 4, "f64", False),
    (2, 2, 2, "p0", 5, "f32", False),
])
def test_gradient_parity_with_oracle(bb, n, N, M, bc, ckpt, dtype, source):
    print(f"[adjoint parity] cube {n} N={N} M={M} {bc} ckpt={ckpt} {dtype} source={source}", flush=True)
    xyz, etov, s, c, q0 = _problem(bb, n, N, M, bc, dtype, 31)
    o = Oracle(xyz, etov, N, M, bc=bc)
    if source:
        g = manufactured_source(c2_sinusoid)
        s.set_source(g, amp=1.5, omega=np.pi)
        o.set_source(g, amp=1.5, omega=np.pi)
    s.set_receivers(PTS)
    rec = Receivers(o, PTS)
    dt, nsteps, t0 = 0.015, 9, 0.05
    data = 0.05 * np.random.default_rng(32).standard_normal((nsteps, len(PTS)))
    if dtype == "f32":  # both sides start from the single-precision state and weight
        q0 = q0.astype(np.float32).astype(np.float64)
        c = c.astype(np.float32).astype(np.float64)
    J, grad, tr = s.misfit_gradient(s.to_device(q0), dt, nsteps, data, checkpoint_every=ckpt, t0=t0)
    Jo, go, tro = misfit_gradient(o, c, o.from_bernstein(q0), dt, nsteps, rec, data, t0=t0)
    g = grad.cpu().numpy()
    tol = 1e-10 if dtype == "f64" else 2e-4
    assert abs(J - Jo) <= tol * abs(Jo), (J, Jo)
    assert np.max(np.abs(tr.cpu().numpy() - tro)) <= tol * np.max(np.abs(tro))
    assert np.max(np.abs(g - go)) <= tol * np.max(np.abs(go)), np.max(np.abs(g - go)) / np.max(np.abs(go))


def test_checkpoint_interval_does_not_change_the_gradient(bb):
    """Recomputing segments from checkpoints reproduces the stored run bit for bit."""
    print("[adjoint checkpoints]", flush=True)
    _, _, s, c, q0 = _problem(bb, 3, 3, 1, "rigid", "f64", 33)
    s.set_receivers(receiver_grid(4, 1.0))
    q = s.to_device(q0)
    data = 0.05 * np.random.default_rng(34).standard_normal((13, 16))
    out = [s.misfit_gradient(q, 0.01, 13, data, checkpoint_every=k) for k in (1, 4, 13, 50)]
    for J, g, tr in out[1:]:
        assert J == out[0][0]
        assert bool((g == out[0][1]).all()) and bool((tr == out[0][2]).all())


def test_adjoint_pairing_identity(bb):
    """(A x, S z)_{L^2} = (x, S B W z)_{L^2} at full precision for random states: the
    transposed operator of the adjoint recursion (B the plain DG operator, W the weighted
    projection, S the velocity reflection)."""
    print("[adjoint pairing]", flush=True)
    xyz, etov = kuhn_cube_mesh(6)
    for bc in ("p0", "rigid"):
        s = bb.Solver(xyz, etov, 4, 2, bc=bc, tau_p=0.7, tau_u=1.3)
        s.set_c2(random_c2_coefficients(35, s.K, s.Mp))
        x = s.to_device(random_state(36, s.K, s.Np))
        z = s.to_device(random_state(37, s.K, s.Np))
        ax, bwz = s.rhs(x), s.adjoint_apply(z)

        def inner(a, b):
            return (s.l2norm2((a + b).contiguous()) - s.l2norm2((a - b).contiguous())) / 4.0

        sign = np.array([1.0, -1.0, -1.0, -1.0])
        lhs = float(np.dot(sign, inner(ax, z)))
        rhs = float(np.dot(sign, inner(x, bwz)))
        # Cauchy-Schwarz bound of the terms, the size of the rounding in both sums
        scale = float(np.sum(np.sqrt(s.l2norm2(ax) * s.l2norm2(z)) + np.sqrt(s.l2norm2(x) * s.l2norm2(bwz))))
        print(f"  {bc}: {lhs!r} {rhs!r} rel {abs(lhs - rhs) / scale:.2e}", flush=True)
        assert abs(lhs - rhs) < 1e-12 * scale, (bc, lhs, rhs)


def test_gradient_matches_central_differences(bb):
    """3,072 tets, N=3, M=1, rigid walls, 16 receivers on the top face, 40 steps; central
    differences of the device's own misfit on 10 random coefficients."""
    print("[adjoint finite differences]", flush=True)
    xyz, etov, s, c, q0 = _problem(bb, 8, 3, 1, "rigid", "f64", 38)
    s.set_receivers(receiver_grid(4, 1.0))
    q = s.to_device(q0)
    dt, nsteps = s.suggest_dt(0.5), 40
    s.set_c2(random_c2_coefficients(39, s.K, s.Mp))  # the "true" medium
    _, _, data = s.misfit_gradient(q, dt, nsteps, None, gradient=False)
    s.set_c2(c)
    J, grad, _ = s.misfit_gradient(q, dt, nsteps, data, checkpoint_every=7)
    g = grad.cpu().numpy()
    rng = np.random.default_rng(40)
    ks = rng.choice(np.nonzero(np.abs(g).max(1) > 1e-3 * np.abs(g).max())[0], 10, replace=False)
    for k in ks:
        b = int(rng.integers(s.Mp))
        h = 1e-4
        cp, cm = c.copy(), c.copy()
        cp[k, b] += h
        cm[k, b] -= h
        s.set_c2(cp)
        jp = s.misfit_gradient(q, dt, nsteps, data, gradient=False)[0]
        s.set_c2(cm)
        jm = s.misfit_gradient(q, dt, nsteps, data, gradient=False)[0]
        fd = (jp - jm) / (2 * h)
        assert abs(fd - g[k, b]) < 1e-6 * np.abs(g).max(), (k, b, fd, g[k, b])


def test_autograd_function_returns_the_adjoint_gradient(bb):
    import torch
    from paper_1808_08645_amd.autograd import c2_misfit
    print("[adjoint autograd]", flush=True)
    _, _, s, c, q0 = _problem(bb, 3, 2, 1, "rigid", "f64", 41)
    s.set_receivers(receiver_grid(3, 1.0))
    q = s.to_device(q0)
    data = torch.zeros((12, 9), dtype=torch.float64, device="cuda")
    c2 = torch.tensor(c, requires_grad=True)
    J = c2_misfit(s, c2, q, 0.01, 12, data, checkpoint_every=5)
    (2.0 * J).backward()
    J0, g0, _ = s.misfit_gradient(q, 0.01, 12, data, checkpoint_every=5)
    assert float(J.detach()) == J0
    assert torch.allclose(c2.grad, 2.0 * g0.cpu(), rtol=0, atol=0)


def test_adjoint_error_paths(bb):
    print("[adjoint errors]", flush=True)
    _, _, s, c, q0 = _problem(bb, 1, 2, 1, "rigid", "f64", 42)
    q = s.to_device(q0)
    with pytest.raises(bb.BBWADGError) as ei:
        s.misfit_gradient(q, 0.01, 3)  # no receivers
    assert ei.value.code == -1
    s.set_receivers([[0.5, 0.5, 0.5]])
    with pytest.raises(bb.BBWADGError):
        s.misfit_gradient(q, 0.01, 0)
    with pytest.raises(bb.BBWADGError):
        s.misfit_gradient(q, 0.01, 3, checkpoint_every=0)
    with pytest.raises(bb.BBWADGError):
        s.misfit_gradient(q, 0.01, 3, np.full((3, 1), np.nan))


def test_full_size_adjoint_pairing_identity(bb):
    """82,944 tets, N=4, M=2 (the adjoint workload's size), rigid walls: the pairing identity
    (A x, S z) = (x, S B W z) in L^2 for random states holds at full size."""
    print("[adjoint pairing full size]", flush=True)
    xyz, etov = kuhn_cube_mesh(24)
    s = bb.Solver(xyz, etov, 4, 2, bc="rigid")
    s.set_c2(random_c2_coefficients(81, s.K, s.Mp))
    x = s.to_device(random_state(82, s.K, s.Np))
    z = s.to_device(random_state(83, s.K, s.Np))
    ax, bwz = s.rhs(x), s.adjoint_apply(z)

    def inner(a, b):
        return (s.l2norm2((a + b).contiguous()) - s.l2norm2((a - b).contiguous())) / 4.0

    sign = np.array([1.0, -1.0, -1.0, -1.0])
    lhs, rhs = float(np.dot(sign, inner(ax, z))), float(np.dot(sign, inner(x, bwz)))
    scale = float(np.sum(np.sqrt(s.l2norm2(ax) * s.l2norm2(z)) + np.sqrt(s.l2norm2(x) * s.l2norm2(bwz))))
    print(f"  rel {abs(lhs - rhs) / scale:.2e}", flush=True)
    assert abs(lhs - rhs) < 1e-12 * scale, (lhs, rhs)
