"""torch.autograd.Function over a checkpointed run of the step.

Differentiable parameters theta = (gamma_01, gamma_02, gamma_12, D^liq_1, D^liq_2, tau)
(pairs and components beyond N and K-1 are ignored) and the initial state.
Forward: mp_step_ckpt; backward: mp_adjoint (hand-written adjoint kernels,
checkpointed recomputation).  dt is held fixed.
"""
from __future__ import annotations

import torch

from . import abi, inputs
from .solver import Solver

THETA_NAMES = ["gamma01", "gamma02", "gamma12", "Dliq1", "Dliq2", "tau"]


def params_with_theta(p, theta):
    """A copy of p with theta written in (theta is a length-6 sequence of floats)."""
    return inputs.theta_into(p, theta)


def theta_of(p):
    N = p.nphases
    g = [float(p.gamma[a, b]) if b < N else 0.0 for a, b in [(0, 1), (0, 2), (1, 2)]]
    d = [float(p.D[N - 1, k]) if k < p.nmu else 0.0 for k in range(2)]
    return g + d + [float(p.tau)]


class PhaseFieldRun(torch.autograd.Function):
    """final_state = run(theta, state0) over nsteps steps, checkpointed every ``every``."""

    @staticmethod
    def forward(ctx, theta, state0, p, nsteps, every):
        q = params_with_theta(p, theta.detach().cpu().tolist())
        s = Solver(q)
        s.bufs[0].copy_(state0.detach().to(s.dtype))
        torch.cuda.synchronize()
        abi.mp_set_step(s.st, 0, 0)
        ckpt = s.checkpoint_buffer(nsteps, every)
        s.step_ckpt(nsteps, every, ckpt)
        out = s.current().clone()
        ctx.solver, ctx.ckpt, ctx.nsteps, ctx.every = s, ckpt, nsteps, every
        ctx.N, ctx.nmu = q.nphases, q.nmu
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        return out

    @staticmethod
    def backward(ctx, grad_out):
        s = ctx.solver
        lam0, g = s.adjoint(grad_out, ctx.ckpt, ctx.nsteps, ctx.every, 0)
        N = ctx.N
        gt = [g["gamma01"], g["gamma02"] if N == 3 else 0.0, g["gamma12"] if N == 3 else 0.0]
        gt += [g[f"D{N - 1}{k}"] if k < ctx.nmu else 0.0 for k in range(2)]
        gt += [g["tau"]]
        s.close()
        ctx.solver = None
        grad_theta = torch.tensor(gt, dtype=ctx.theta_dtype, device=ctx.theta_device)
        return grad_theta, lam0, None, None, None


def run(theta, state0, p, nsteps, every):
    return PhaseFieldRun.apply(theta, state0, p, nsteps, every)
