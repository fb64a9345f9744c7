"""Host-side pieces of the surrogate-assisted inversion: the linear maps from the medium
parameters to the solver's c^2 coefficients and to the surrogate's input, and the pull-back
of an input gradient (the transpose of the input map)."""
import numpy as np
import pytest

from paper_1808_08645_amd.inversion import LinearMedium, _adam
from workloads import c2_random_model, c2_random_model_family, grid_centres


class _FakeSolver:
    """project_function samples phi at fixed points: linear in phi, as the real projection is."""
    M = 2

    def __init__(self, K=7, Mp=10, seed=0):
        rng = np.random.default_rng(seed)
        self.pts = rng.uniform(0, 1, size=(K, Mp, 3))

    def project_function(self, fn, degree):
        assert degree == self.M
        return np.asarray(fn(self.pts[..., 0], self.pts[..., 1], self.pts[..., 2]), dtype=np.float64)


def _medium(seed=3):
    phis, theta = c2_random_model_family(seed)
    return LinearMedium(_FakeSolver(), phis, grid_centres(16)), theta, phis


def test_family_reproduces_the_model():
    # sum_i theta_i phi_i is the model before clipping; where it lies in [1, 4] they agree
    phis, theta = c2_random_model_family(5)
    x, y, z = grid_centres(16)
    lin = sum(t * phi(x, y, z) for t, phi in zip(theta, phis))
    ref = c2_random_model(5)(x, y, z)
    inside = (lin > 1.0) & (lin < 4.0)
    assert inside.mean() > 0.5
    np.testing.assert_allclose(lin[inside], ref[inside], rtol=0, atol=1e-12)


def test_coef_is_linear_and_differentiable():
    import torch
    med, theta, phis = _medium()
    c = med.coef(theta)
    direct = sum(t * med.solver.project_function(phi, 2) for t, phi in zip(theta, phis))
    np.testing.assert_allclose(c, direct, rtol=1e-13, atol=1e-13)
    th = torch.tensor(theta, requires_grad=True)
    ct = med.coef(th)
    np.testing.assert_allclose(ct.detach().numpy(), c, rtol=1e-13, atol=1e-13)
    w = torch.tensor(np.random.default_rng(1).standard_normal(c.shape))
    (ct * w).sum().backward()
    expect = np.array([(med.solver.project_function(phi, 2) * w.numpy()).sum() for phi in phis])
    np.testing.assert_allclose(th.grad.numpy(), expect, rtol=1e-12)


def test_input_gradient_pull_back_is_the_transpose():
    med, theta, phis = _medium()
    rng = np.random.default_rng(2)
    G = rng.standard_normal((16, 16, 16))
    g = med.theta_grad_from_input(G)
    # <x(theta + d) - x(theta), G> = <d, g> for the affine input map (float32 inputs)
    for _ in range(3):
        d = rng.standard_normal(theta.shape) * 0.1
        lhs = float(np.sum((med.grid_input(theta + d)[0].astype(np.float64) - med.grid_input(theta)[0]) * G))
        assert abs(lhs - float(d @ g)) <= 1e-5 * max(1.0, abs(lhs))
    # and against the definition: x = (sum theta_i phi_i(grid) - shift) / scale
    x, y, z = grid_centres(16)
    xin = (sum(t * phi(x, y, z) for t, phi in zip(theta, phis)) - 2.5) / 1.5
    np.testing.assert_allclose(med.grid_input(theta)[0], xin, rtol=1e-6, atol=1e-6)


def test_adam_first_step_moves_by_lr_against_the_sign():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -0.1, 0.0])
    th, state = _adam(theta, g, (np.zeros(3), np.zeros(3), 0), lr=0.01)
    np.testing.assert_allclose(th, theta - 0.01 * np.sign(g) * (np.abs(g) / (np.abs(g) + 1e-8)), rtol=1e-12)
    assert state[2] == 1


@pytest.mark.parametrize("seed", [0, 1])
def test_grid_input_range(seed):
    med, theta, _ = _medium(seed)
    x = med.grid_input(theta)
    assert x.shape == (1, 16, 16, 16) and x.dtype == np.float32
