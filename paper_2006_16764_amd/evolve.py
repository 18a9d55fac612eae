"""Checkpointed backward-Euler evolution as a torch.autograd.Function.

Forward: pf_evolve runs the Newton-Krylov steps U^1..U^K from U^0 and keeps
every state (the checkpoints).  Backward: the discrete adjoint of the stepping,
one pf_adjoint_step per step from K down to 1, gives dL/d eps4, dL/d lambda and
dL/dU^0 for a loss of U^K.  The misfit L = 1/2 sum_i m_i (phi_i^K - phi*_i)^2
(lumped nodal mass m_i) is a second Function over pf_misfit.

Everything on the data is done by the library; this module only moves
pointers, shapes and scalars.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import binding


class PhaseFieldEvolve(torch.autograd.Function):
    """U^K = evolve(eps4, lam, U^0) over `steps` backward-Euler steps."""

    @staticmethod
    def forward(ctx, eps4: torch.Tensor, lam: torch.Tensor, U0: torch.Tensor,
                problem: binding.Problem, steps: int, opts: Optional[binding.pf_solver_opts] = None):
        o = opts if opts is not None else binding.default_opts()
        p = problem.params
        if p.theta != 1.0:
            raise ValueError("the adjoint covers backward Euler (theta = 1) only")
        params = binding.make_params(p.dim, list(p.n)[:p.dim], list(p.half_width)[:p.dim], p.dt,
                                     float(eps4), float(lam), p.D, p.delta2, p.theta)
        problem.set_params(params)
        n = problem.n_dof
        states = torch.empty((steps + 1) * n, dtype=torch.float64, device=U0.device)
        states[:n].copy_(U0.reshape(-1))
        stats = problem.pf_evolve(states, steps, o)
        ctx.problem, ctx.steps, ctx.opts, ctx.params = problem, steps, o, params
        ctx.stats = stats
        ctx.save_for_backward(states)
        return states[steps * n:].clone()

    @staticmethod
    def backward(ctx, grad_UK: torch.Tensor):
        (states,) = ctx.saved_tensors
        pb, K, o = ctx.problem, ctx.steps, ctx.opts
        pb.set_params(ctx.params)
        n = pb.n_dof
        S = states.view(K + 1, n)
        # a copy: the two adjoint buffers are swapped and overwritten step by
        # step, and the incoming gradient belongs to the caller
        mu = grad_UK.reshape(-1).to(torch.float64).clone()
        lam, mu_prev = pb.new_vector(), pb.new_vector()
        gp = torch.zeros(2, dtype=torch.float64, device=states.device)
        for k in range(K, 0, -1):
            pb.pf_adjoint_step(S[k], S[k - 1], mu, lam, mu_prev, gp, o)
            mu, mu_prev = mu_prev, mu
        return gp[0], gp[1], mu.view_as(grad_UK), None, None, None


class PhaseFieldMisfit(torch.autograd.Function):
    """L = 1/2 sum_i m_i (phi_i - phi*_i)^2 of an interleaved state U."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, phi_target: torch.Tensor, problem: binding.Problem):
        L = torch.zeros(1, dtype=torch.float64, device=U.device)
        g = problem.new_vector()
        problem.pf_misfit(U.reshape(-1).contiguous(), phi_target.contiguous(), L, g)
        ctx.save_for_backward(g)
        return L[0]

    @staticmethod
    def backward(ctx, grad_L: torch.Tensor):
        (g,) = ctx.saved_tensors
        return g * grad_L, None, None


def evolve(eps4, lam, U0, problem, steps, opts=None):
    return PhaseFieldEvolve.apply(eps4, lam, U0, problem, steps, opts)


def misfit(U, phi_target, problem):
    return PhaseFieldMisfit.apply(U, phi_target, problem)
