"""Autograd front end of form (3): gradients of any loss of the forces and
per-box energies with respect to the B-spline coefficients of V(r), rho(r)
and F(rho).  Forward runs md_set_theta + md_forces; backward runs the
hand-written adjoint kernel (md_adjoint).  Argument marshalling only."""
from __future__ import annotations

import torch


class SplineEAMFunction(torch.autograd.Function):
    """(theta_phi, theta_f, theta_F, system) -> (forces [N, 3], box energies [B]).

    `system` is an md.System created with a B-spline potential whose state
    (positions) has been set.  The coefficients are float64 CUDA tensors of
    equal length K.
    """

    @staticmethod
    def forward(ctx, theta_phi, theta_f, theta_F, system):
        theta = torch.cat([theta_phi.reshape(-1), theta_f.reshape(-1),
                           theta_F.reshape(-1)]).to(torch.float64).contiguous()
        system.set_theta(theta)
        f, _, eb = system.forces(energy=True)
        ctx.system = system
        ctx.K = theta_phi.numel()
        ctx.save_for_backward(theta)
        return f, eb

    @staticmethod
    def backward(ctx, g_f, g_e):
        S = ctx.system
        (theta,) = ctx.saved_tensors
        S.set_theta(theta)
        if g_f is None:
            g_f = torch.zeros(S.n_atoms, 3, dtype=torch.float64, device=theta.device)
        if g_e is None:
            g_e = torch.zeros(S.n_boxes, dtype=torch.float64, device=theta.device)
        gt = S.adjoint(g_f.contiguous(), g_e.contiguous())
        K = ctx.K
        return gt[:K], gt[K:2 * K], gt[2 * K:], None


def force_matching_loss(system, theta_phi, theta_f, theta_F, f_target, e_target, w):
    """sum |f - f_target|^2 + w sum_b (E_b - E_target_b)^2."""
    f, eb = SplineEAMFunction.apply(theta_phi, theta_f, theta_F, system)
    return ((f - f_target) ** 2).sum() + w * ((eb - e_target) ** 2).sum()
