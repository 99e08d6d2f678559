"""torch.autograd.Functions over the hand-written adjoints.

LogKMisfit.apply(logk0, problem) runs one linear Picard stage from the
problem's initial state with k0 = exp(logk0) and returns the sensor misfit
J = 1/2 sum_s (Pf_s - d_s)^2; the stage adjoint (pt_adjoint_stage) runs with
the forward and backward returns its dJ/d(logk0).

LogKMisfitRun.apply(logk0, run_problem) does the same for a run of Picard
steps x stages (pt_adjoint_run: recorded forward, then the reverse sweep; the
gradient is computed with the forward and kept for backward).

Every step runs in the HIP library.
"""
from __future__ import annotations

import torch


class StageProblem:
    """A Grid plus the data of one linear-stage misfit problem."""

    def __init__(self, grid, phi, sensors, d_obs, rtol=1e-12, max_iter=2_000_000):
        self.grid = grid
        self.phi = phi
        self.sensors = sensors
        self.d_obs = d_obs
        self.rtol = rtol
        self.max_iter = max_iter

    def forward(self, logk0) -> float:
        g = self.grid
        g.reset_state(self.phi)
        g.set_log_k0(logk0)
        g.begin_step(False)
        g.refresh(1.0, 1.0)
        it, rho, ok = g.solve_linear(self.rtol, self.max_iter)
        if not ok:
            raise RuntimeError(f"stage solve did not reach rtol {self.rtol} (rho {rho:.3e})")
        return g.misfit(self.sensors, self.d_obs)


class LogKMisfit(torch.autograd.Function):
    """The gradient is computed with the forward (the stage adjoint needs the
    grid in the state the forward left, which a later forward on the same
    problem would overwrite) and kept for backward."""

    @staticmethod
    def forward(ctx, logk0: torch.Tensor, problem: StageProblem):
        J = problem.forward(logk0.detach())
        p = problem
        _J, grad, _it, _rho, ok = p.grid.adjoint_stage(p.sensors, p.d_obs, p.rtol, p.max_iter)
        if not ok:
            raise RuntimeError("adjoint solve did not converge")
        ctx.save_for_backward(grad.clone())
        return logk0.new_tensor(J)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None


class RunProblem:
    """A Grid plus the data of a Picard-run misfit problem."""

    def __init__(self, grid, phi, sensors, d_obs, n_steps, n_picard, rtol=1e-11, adj_rtol=None,
                 max_iter=2_000_000, checkpoint=False):
        self.grid = grid
        self.phi = phi
        self.sensors = sensors
        self.d_obs = d_obs
        self.n_steps = n_steps
        self.n_picard = n_picard
        self.rtol = rtol
        self.adj_rtol = rtol if adj_rtol is None else adj_rtol
        self.max_iter = max_iter
        self.checkpoint = checkpoint

    def forward(self, logk0):
        """(J, dJ/dlogk0 as a new device tensor) of the run from the initial state."""
        g = self.grid
        g.reset_state(self.phi)
        g.set_log_k0(logk0)
        J, grad, _fit, _ait = g.adjoint_run(self.sensors, self.d_obs, self.n_steps, self.n_picard, self.rtol,
                                            self.adj_rtol, self.max_iter, self.checkpoint)
        return J, grad.clone()


class LogKMisfitRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logk0: torch.Tensor, problem: RunProblem):
        J, grad = problem.forward(logk0.detach())
        ctx.save_for_backward(grad)
        return logk0.new_tensor(J)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None
