"""Inversion of the receiver misfit for c^2 over a few medium parameters, with the trace
surrogate standing in for the forward solve and BBWADG as its check and fallback.

The medium is linear in its parameters, c^2(x; theta) = sum_i theta_i phi_i(x), so both the
weight the solver takes (the degree-M projection of c^2, a Bernstein coefficient array) and
the surrogate's input (c^2 at the cell centres of its grid) are linear maps of theta, and
gradients come back to theta through their transposes:

* BBWADG: J(theta) = c2_misfit(solver, Psi^T theta) (the autograd wrapper of the
  checkpointed discrete adjoint), so J.backward() leaves dJ/dtheta in theta.grad;
* surrogate: J_S(theta) = 1/2 sum (sigma f(x(theta)) - d)^2 with x the normalised grid input;
  its gradient is the network's input gradient pulled back through the grid map.

The rule that decides between them runs with the loop, from BBWADG's own runs: a
surrogate round takes `inner` Adam steps on J_S and is then checked by one BBWADG forward run
at the new theta. The round is kept when the true misfit fell and the surrogate's relative
trace error at that theta is at most `max_err`. A round whose traces were within `max_err`
but whose misfit did not fall is retried from the kept theta with a quarter of the step
size (the surrogate is trusted there, its step was too long), at most `retries` times in a
row; a round whose trace error exceeds `max_err`, or the last allowed retry, leaves theta
where it was and hands the rest of the run to BBWADG gradient steps (backtracking on the
true misfit).
"""
from __future__ import annotations

import time

import numpy as np


class LinearMedium:
    """c^2(x; theta) = sum_i theta_i phi_i(x) on a solver's mesh and on the surrogate grid.

    ``grid_xyz`` holds the surrogate's input points (x, y, z arrays of its grid shape);
    inputs are normalised as (c^2 - x_shift) / x_scale, the normalisation the surrogate was
    trained with."""

    def __init__(self, solver, phis, grid_xyz, x_shift: float = 2.5, x_scale: float = 1.5):
        import torch
        self.solver = solver
        self.phis = list(phis)
        # Bernstein coefficients of the degree-M projection of each phi_i: [n][K][Mp]
        psi = np.stack([solver.project_function(phi, solver.M) for phi in self.phis])
        self.Psi = torch.as_tensor(psi, dtype=torch.float64)
        gx, gy, gz = grid_xyz
        self.Phi = np.stack([np.asarray(phi(gx, gy, gz), dtype=np.float64) for phi in self.phis])
        self.x_shift, self.x_scale = float(x_shift), float(x_scale)

    @property
    def n(self) -> int:
        return len(self.phis)

    def coef(self, theta):
        """Projected c^2 coefficients [K][Mp]; a torch tensor when theta is one (keeps autograd)."""
        import torch
        if isinstance(theta, torch.Tensor):
            return torch.tensordot(theta.to(torch.float64), self.Psi, 1)
        return np.tensordot(np.asarray(theta, dtype=np.float64), self.Psi.numpy(), 1)

    def grid_input(self, theta) -> np.ndarray:
        """The surrogate's normalised input [1][g][g][g] (float32) for theta."""
        c2 = np.tensordot(np.asarray(theta, dtype=np.float64), self.Phi, 1)
        return ((c2 - self.x_shift) / self.x_scale).astype(np.float32)[None]

    def theta_grad_from_input(self, g_x) -> np.ndarray:
        """Pull dJ/dx (one input, grid-shaped) back to dJ/dtheta."""
        g = np.asarray(g_x, dtype=np.float64).reshape(self.Phi.shape[1:])
        return np.tensordot(self.Phi, g, axes=(list(range(1, self.Phi.ndim)), list(range(g.ndim)))) / self.x_scale


def _adam(theta, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    m, v, k = state
    k += 1
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh, vh = m / (1 - b1 ** k), v / (1 - b2 ** k)
    return theta - lr * mh / (np.sqrt(vh) + eps), (m, v, k)


class Inversion:
    """Minimise J(theta) = 1/2 sum_{n,r} (p(x_r, t_n; theta) - d_{n,r})^2 over theta.

    ``surrogate`` (a trained Surrogate whose outputs are the traces divided by ``sigma``,
    flattened as [nsteps * nrec]) enables the surrogate rounds; without it every iteration
    is a BBWADG gradient step."""

    def __init__(self, solver, medium: LinearMedium, q0, dt: float, nsteps: int, data, surrogate=None,
                 sigma: float = 1.0, checkpoint_every: int = 50):
        import torch
        self.s, self.med, self.q0, self.dt, self.nsteps = solver, medium, q0, float(dt), int(nsteps)
        self.data = torch.as_tensor(np.asarray(data), dtype=torch.float64, device="cuda").contiguous()
        self.sur, self.sigma, self.ckpt = surrogate, float(sigma), int(checkpoint_every)
        self.target = None
        if surrogate is not None:
            t = (np.asarray(data, dtype=np.float64).reshape(1, -1) / self.sigma).astype(np.float32)
            self.target = torch.as_tensor(t, device="cuda")
        self.forward_runs = 0
        self.gradient_runs = 0

    def _valid(self, theta) -> bool:
        import paper_1808_08645_amd as bb
        try:
            self.s.set_c2(self.med.coef(theta))
            return True
        except bb.BBWADGError:  # c^2_M not positive everywhere: not a valid medium
            return False

    def misfit(self, theta):
        """One BBWADG forward run: (J, traces), or (inf, None) for an invalid medium."""
        import torch
        if not self._valid(theta):
            return np.inf, None
        J, _, tr = self.s.misfit_gradient(self.q0, self.dt, self.nsteps, self.data, self.ckpt, gradient=False)
        torch.cuda.synchronize()
        self.forward_runs += 1
        return J, tr

    def gradient(self, theta):
        """BBWADG misfit and dJ/dtheta through autograd (forward run, then the adjoint)."""
        import torch

        from .autograd import c2_misfit
        th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
        if not self._valid(theta):
            raise ValueError("gradient requested at an invalid medium")
        J = c2_misfit(self.s, self.med.coef(th), self.q0, self.dt, self.nsteps, self.data, self.ckpt)
        J.backward()
        torch.cuda.synchronize()
        self.gradient_runs += 1
        return float(J.detach()), th.grad.numpy().copy()

    def surrogate_misfit_grad(self, theta):
        """(J_S, dJ_S/dtheta) in the units of J: J_S = sigma^2 nout / 2 * mean((f - d/sigma)^2)."""
        loss, dx = self.sur.input_grad(self.med.grid_input(theta), self.target)
        scale = self.sigma ** 2 * self.sur.nout / 2.0
        return scale * loss, scale * self.med.theta_grad_from_input(dx.cpu().numpy()[0])

    def surrogate_error(self, theta, traces) -> float:
        """Relative L2 error of the surrogate's traces against BBWADG's at theta."""
        y = self.sur.forward(self.med.grid_input(theta)).double().cpu().numpy().ravel() * self.sigma
        t = traces.cpu().numpy().ravel()
        return float(np.linalg.norm(y - t) / max(np.linalg.norm(t), 1e-300))

    def run(self, theta0, max_time: float = 60.0, target: float = 0.0, inner: int = 40, lr: float = 0.02,
            max_err: float = 0.2, step0: float = 0.2, max_iters: int = 1000, retries: int = 2):
        """Iterate until J <= target * J(theta0), max_time seconds or max_iters iterations.
        Returns (theta, history); each history entry has the wall time t, the kept misfit J
        and what the iteration was."""
        theta = np.asarray(theta0, dtype=np.float64).copy()
        t0 = time.perf_counter()
        J, _ = self.misfit(theta)
        J0 = J
        hist = [{"t": 0.0, "J": J, "kind": "start"}]
        mode = "surrogate" if self.sur is not None else "bbwadg"
        zero = (np.zeros_like(theta), np.zeros_like(theta), 0)
        adam, lr_s, misses = zero, lr, 0
        for _ in range(max_iters):
            if time.perf_counter() - t0 >= max_time or J <= target * J0:
                break
            if mode == "surrogate":
                th, st = theta.copy(), adam
                for _ in range(inner):
                    _, g = self.surrogate_misfit_grad(th)
                    th, st = _adam(th, g, st, lr_s)
                Jn, trn = self.misfit(th)
                err = self.surrogate_error(th, trn) if trn is not None else np.inf
                ok = bool(Jn < J and err <= max_err)
                hist.append({"t": time.perf_counter() - t0, "J": Jn if ok else J, "kind": "surrogate round",
                             "accepted": ok, "surrogate_err": err, "J_tried": float(Jn), "lr": lr_s})
                if ok:
                    theta, J, adam, misses = th, Jn, st, 0
                elif err <= max_err and misses < retries:
                    misses += 1
                    lr_s, adam = lr_s / 4.0, zero
                else:
                    mode = "bbwadg"
                continue
            Jg, g = self.gradient(theta)
            gn = float(np.max(np.abs(g)))
            if gn == 0.0:
                break
            alpha = step0 / gn
            while True:
                th = theta - alpha * g
                Jn, _ = self.misfit(th)
                if Jn < J or alpha * gn < 1e-4:
                    break
                alpha *= 0.5
            improved = Jn < J
            if improved:
                theta, J = th, Jn
            hist.append({"t": time.perf_counter() - t0, "J": J, "kind": "bbwadg gradient step", "alpha": alpha})
            if not improved:
                break
        return theta, hist
