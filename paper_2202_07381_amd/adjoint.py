"""Differentiable IRK time stepping on top of the C ABI.

``IrkSteps`` runs N steps of the IRK scheme (right-hand side, FGMRES solve of the
stage system preconditioned by the Vanka V-cycle, update) and keeps every step's state
and stages on the device (the checkpoints).  Its backward pass is the discrete adjoint:
for n = N-1 .. 0 it solves J^T lam = dt b (x) gbar with FGMRES preconditioned by the
transposed V-cycle (``irk_adjoint_solve``), maps lam back to the forcing and the state
(``irk_rhs_adjoint``, adding into the state adjoint in place) and adds the viscosity
sensitivity of the step (``irk_nu_sensitivity``, accumulating into one device value).
``tracking_loss`` is 1/2 (u - u_hat)^T M (u - u_hat) (``irk_tracking_loss``, which also
gives both gradients scaled by the incoming gradient).  All arithmetic runs in the
library; this module only allocates tensors and sequences calls.
"""
from __future__ import annotations

import torch

from .irkmg import IrkMG


class IrkSteps(torch.autograd.Function):
    """state_N = IrkSteps.apply(f_all, nu, state0, solver, rtol, maxit).

    f_all:  (nsteps, r, nnodes, dim) float64 CUDA tensor, nodal forcing of every stage
            of every step on the finest level (node numbering of the C ABI).
    nu:     0-d float64 tensor equal to the viscosity the solver was set up with
            (only its gradient is produced here).
    state0: (ns,) float64 CUDA tensor, the initial (u, p) in the stage-block layout.
    """

    @staticmethod
    def forward(ctx, f_all, nu, state0, solver: IrkMG, rtol: float = 1e-10, maxit: int = 500):
        if abs(float(nu) - solver.nu) > 1e-15 * max(1.0, abs(solver.nu)):
            raise ValueError("nu must equal the viscosity the solver was built with")
        N = solver.irk_mg_ndofs()
        state = state0.detach().clone().contiguous()
        saved, its = [], []
        F = torch.empty(N, dtype=torch.float64, device=state.device)
        for n in range(f_all.shape[0]):
            k = torch.zeros(N, dtype=torch.float64, device=state.device)
            solver.irk_rhs(f_all[n].contiguous().view(-1), state, F)
            info = solver.irk_fgmres_solve(F, k, rtol=rtol, maxit=maxit, history_cap=0)
            if not info["converged"]:
                raise RuntimeError(f"forward solve of step {n} did not converge: {info}")
            its.append(info["iterations"])
            saved += [state.clone(), k]
            solver.irk_update(k, state)
        ctx.save_for_backward(*saved)
        ctx.solver, ctx.rtol, ctx.maxit = solver, rtol, maxit
        ctx.fshape = f_all.shape
        ctx.forward_iterations = its
        return state

    @staticmethod
    def backward(ctx, g_state):
        solver: IrkMG = ctx.solver
        saved = ctx.saved_tensors
        nsteps = len(saved) // 2
        N = solver.irk_mg_ndofs()
        dev = g_state.device
        gbar = g_state.detach().clone().contiguous()
        gf = torch.empty(ctx.fshape, dtype=torch.float64, device=dev)
        gnu = torch.zeros(1, dtype=torch.float64, device=dev)
        G = torch.empty(N, dtype=torch.float64, device=dev)
        for n in range(nsteps - 1, -1, -1):
            state_n, k_n = saved[2 * n], saved[2 * n + 1]
            solver.irk_update_adjoint(gbar, G)
            lam = torch.zeros(N, dtype=torch.float64, device=dev)
            info = solver.irk_adjoint_solve(G, lam, rtol=ctx.rtol, maxit=ctx.maxit, history_cap=0)
            if not info["converged"]:
                raise RuntimeError(f"adjoint solve of step {n} did not converge: {info}")
            # gbar_n = gbar_{n+1} + (dF/dstate)^T lam^n, gnu += lam^nT (dF/dnu - dJ/dnu k^n)
            solver.irk_rhs_adjoint(lam, gf[n].view(-1), gbar, accumulate=True)
            solver.irk_nu_sensitivity(lam, k_n, state_n, gnu, accumulate=True)
        return gf, gnu.view(()), gbar, None, None, None


class TrackingLoss(torch.autograd.Function):
    """L = 1/2 (u - u_hat)^T M (u - u_hat) over the velocity part of a state."""

    @staticmethod
    def forward(ctx, state, target, solver: IrkMG):
        state, target = state.detach().contiguous(), target.detach().contiguous()
        loss = torch.empty(1, dtype=torch.float64, device=state.device)
        solver.irk_tracking_loss(state, target, loss=loss)
        ctx.save_for_backward(state, target)
        ctx.solver = solver
        return loss.view(())

    @staticmethod
    def backward(ctx, g):
        state, target = ctx.saved_tensors
        gs, gt = torch.empty_like(state), torch.empty_like(target)
        scale = g.detach().to(dtype=torch.float64).reshape(1).contiguous()
        ctx.solver.irk_tracking_loss(state, target, grad_state=gs, grad_target=gt, scale=scale)
        return gs, gt, None


def tracking_loss(state, target, solver: IrkMG):
    return TrackingLoss.apply(state, target, solver)
