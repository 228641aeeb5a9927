"""torch.autograd wrapper of the recorded forward pass and its hand-written adjoint.

``flow_velocity(phi, ...)`` runs ``steps`` collide-and-stream cycles of the
porous MRT-LB scheme on the GPU from the rest state and returns u(T) as a
[2, ny, nx] tensor; ``loss.backward()`` then calls the library's discrete
adjoint (lbm_backward / lbm_backward_params) with checkpointed
recomputation, so gradients reach the porosity field, the 1/K field (with a
kappa plane) and the scalar parameters (nu, a_x, a_y, lid velocity). Argument
marshalling only: the forward and backward passes run in the HIP library.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import lbm

THETA_NAMES = ("nu", "ax", "ay", "lid_ux")


class _FlowVelocity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, kappa, theta, desc, steps, ckpt_every):
        d = lbm.Desc.from_buffer_copy(desc)
        if theta is not None:
            vals = [float(v) for v in theta.detach().cpu().tolist()]
            d.nu, d.ax, d.ay, d.lid_ux = vals
        d.ckpt_every = int(ckpt_every)
        solver = lbm.Solver(d, phi=None if phi is None else phi.detach().contiguous(),
                            kappa=None if kappa is None else kappa.detach().contiguous(),
                            max_steps_recorded=int(steps), device=phi.device if phi is not None else "cuda")
        solver.step(int(steps))
        _, u, _ = solver.macroscopic()
        ctx.solver = solver
        ctx.has_phi = phi is not None
        ctx.has_kappa = kappa is not None
        ctx.theta_meta = None if theta is None else (theta.dtype, theta.device)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        s = ctx.solver
        want_phi = ctx.has_phi and ctx.needs_input_grad[0]
        want_kappa = ctx.has_kappa and ctx.needs_input_grad[1]
        want_theta = ctx.theta_meta is not None and ctx.needs_input_grad[2]
        g_phi = g_kappa = g_theta = None
        if want_theta:
            gp, gk, th = s.backward_params(grad_u.contiguous(), want_phi=want_phi, want_kappa=want_kappa)
            dtype, device = ctx.theta_meta
            g_theta = torch.tensor([th[n] for n in THETA_NAMES], dtype=dtype, device=device)
            g_phi, g_kappa = gp, gk
        elif want_phi or want_kappa:
            g_phi, g_kappa = s.backward(grad_u.contiguous(), want_kappa=want_kappa)
            if not want_phi:
                g_phi = None
        ctx.solver = None
        return g_phi, g_kappa, g_theta, None, None, None


def flow_velocity(phi: Optional[torch.Tensor], desc: lbm.Desc, steps: int, ckpt_every: int = 200,
                  kappa: Optional[torch.Tensor] = None, theta: Optional[torch.Tensor] = None) -> torch.Tensor:
    """u(T) [2, ny, nx] after ``steps`` cycles from the rest state, differentiable with
    respect to phi [ny, nx] (the medium's porosity plane), kappa [ny, nx] (1/K, with
    MEDIUM_PHI_KAPPA) and theta = (nu, a_x, a_y, lid_ux) (overrides desc's values).
    Checkpoints every ``ckpt_every`` cycles bound the recording's memory."""
    return _FlowVelocity.apply(phi, kappa, theta, desc, int(steps), int(ckpt_every))


def outlet_flow(phi: Optional[torch.Tensor], desc: lbm.Desc, steps: int, ckpt_every: int = 200,
                kappa: Optional[torch.Tensor] = None, theta: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The outlet profile u(T)[:, :, nx - 1] as a [2, ny] tensor (the sensor column of the
    inverse problem), differentiable like ``flow_velocity``: its gradient reaches the adjoint
    as dL/du that is zero off the outlet column."""
    return flow_velocity(phi, desc, steps, ckpt_every, kappa=kappa, theta=theta)[:, :, -1]
