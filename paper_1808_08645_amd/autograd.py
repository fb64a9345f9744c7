"""The receiver misfit as a differentiable function of the c^2_M Bernstein coefficients.

``c2_misfit(solver, c2, q0, dt, nsteps, data)`` returns J(c2) as a 0-d tensor; its backward
pass calls the library's checkpointed discrete adjoint (bbwadg_misfit_gradient), so
``J.backward()`` leaves dJ/dc2 in ``c2.grad``. The forward pass runs the forward solve only.
"""
import torch


class C2Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c2, solver, q0, dt, nsteps, data, checkpoint_every, t0):
        solver.set_c2(c2.detach().to("cpu", torch.float64).numpy())
        J, _, _ = solver.misfit_gradient(q0, dt, nsteps, data, checkpoint_every, t0, gradient=False)
        ctx.args = (solver, q0, dt, nsteps, data, checkpoint_every, t0)
        ctx.c2_meta = (c2.dtype, c2.device)
        ctx.save_for_backward(c2)
        return torch.tensor(J, dtype=torch.float64, device=c2.device)

    @staticmethod
    def backward(ctx, gJ):
        (c2,) = ctx.saved_tensors
        solver, q0, dt, nsteps, data, checkpoint_every, t0 = ctx.args
        solver.set_c2(c2.detach().to("cpu", torch.float64).numpy())  # the solver may have moved on
        _, grad, _ = solver.misfit_gradient(q0, dt, nsteps, data, checkpoint_every, t0, gradient=True)
        dtype, device = ctx.c2_meta
        g = (grad * gJ.to(grad.device)).to(device=device, dtype=dtype)
        return g, None, None, None, None, None, None, None


def c2_misfit(solver, c2, q0, dt, nsteps, data, checkpoint_every=50, t0=0.0):
    return C2Misfit.apply(c2, solver, q0, dt, nsteps, data, checkpoint_every, t0)
