"""Receiver-misfit gradients through the library's discrete adjoint.

MisfitProblem fixes everything but the material: mesh, degree, precision,
reference fields rho, lambda, mu at the quadrature points, source,
receivers, observed traces, dt and step count.  Its parameters are
per-element multipliers theta [K][3] of the reference fields (theta = 1 is
the reference medium).  MisfitFn wraps it as a torch.autograd.Function:
forward runs ewdg_forward_misfit (forward solve with checkpoints, J on the
receiver traces), backward runs ewdg_adjoint_gradient (checkpointed reverse
sweep of the transposed stages).

The library differentiates with respect to multipliers s applied on top of
the material it holds (s = 1); with that material equal to reference *
theta, dJ/dtheta = (dJ/ds) / theta element- and field-wise.
"""
import numpy as np
import torch

from . import ewdg as B


class MisfitProblem:
    def __init__(self, N, EToV, VXYZ, rho_q, lam_q, mu_q, source, receivers, data, dt, nsteps,
                 precision=32, checkpoint_every=50, q0=None, t0=0.0, stream=None):
        """source: (xs, direction, amp, f0, t0_ricker); receivers [nr][3];
        data [nsteps][nr][3]; q0 the initial state (zero if None)."""
        self.ctx = B.Context(N, precision, stream=stream)
        self.ctx.set_mesh(EToV, VXYZ)
        self.receivers = np.asarray(receivers, dtype=np.float64).reshape(-1, 3)
        self.nsteps = int(nsteps)
        self.ctx.bind_workspace(self.receivers.shape[0], self.nsteps)
        self.ctx.bind_adjoint_workspace(self.nsteps, checkpoint_every)
        self.base = [np.asarray(x, dtype=np.float64).reshape(self.ctx.K, self.ctx.Nq) for x in (rho_q, lam_q, mu_q)]
        self.source = source
        self.data = np.asarray(data, dtype=np.float64).reshape(self.nsteps, self.receivers.shape[0], 3)
        self.dt = float(dt)
        self.q0 = q0
        self.t0 = float(t0)
        self.theta = None
        self.K = self.ctx.K

    def _set_theta(self, theta):
        th = np.asarray(theta, dtype=np.float64).reshape(self.K, 3)
        if not np.all(th > 0):
            raise ValueError("multipliers must be positive")
        mats = [b * th[:, k:k + 1] for k, b in enumerate(self.base)]
        c = self.ctx
        c.set_material(*mats)
        xs, d, amp, f0, tr = self.source
        c.set_source(xs, d, amp, f0, tr)
        if self.receivers.shape[0]:
            c.set_receivers(self.receivers)
        if self.q0 is None:
            c.set_state(torch.zeros((self.K, 9, c.Np), dtype=c.torch_dtype, device="cuda"), self.t0)
        else:
            c.set_state(self.q0, self.t0)
        self.theta = th

    def misfit(self, theta):
        """J(theta); records the run for gradient()."""
        self._set_theta(theta)
        return self.ctx.forward_misfit(self.dt, self.nsteps, self.data)

    def gradient(self):
        """dJ/dtheta [K][3] (FP64, device) of the last misfit() call."""
        g, _ = self.ctx.adjoint_gradient()
        return g / torch.as_tensor(self.theta, device=g.device)

    def traces(self):
        return self.ctx.receivers()

    def close(self):
        self.ctx.close()


class MisfitFn(torch.autograd.Function):
    """J = MisfitFn.apply(theta, problem): theta [K][3] tensor of per-element
    multipliers (rho, lambda, mu) of the problem's reference fields."""

    @staticmethod
    def forward(ctx, theta, problem):
        th = theta.detach().cpu().numpy().astype(np.float64)
        J = problem.misfit(th)
        ctx.problem = problem
        ctx.theta_key = th.reshape(problem.K, 3).copy()
        return torch.tensor(J, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        p = ctx.problem
        if p.theta is None or not np.array_equal(p.theta, ctx.theta_key):
            raise RuntimeError("the problem ran another misfit since this forward; run it again")
        g = p.gradient().to(grad_out.device)
        return (grad_out * g).to(dtype=grad_out.dtype), None
