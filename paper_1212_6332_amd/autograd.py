"""Autograd front end of form (3): gradients of any loss of the forces and
per-box energies with respect to the B-spline coefficients of V(r), rho(r)
and F(rho).  Forward runs md_set_theta + md_forces; backward runs the
hand-written adjoint kernel (md_adjoint).  Argument marshalling only.

GraphedLoss captures one loss evaluation with its backward pass in a HIP
graph (through torch.cuda.graph) and replays it, which removes the host cost
of the Python autograd engine and of some thirty launches per evaluation."""
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
        f, _, eb = system.forces(energy=True, atom_energy=False)
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


class GraphedLoss:
    """A loss of the forces and energies and its backward pass, captured once
    in a HIP graph and replayed.

    `loss_fn()` returns a scalar loss computed from the leaf tensors `params`
    (float64 CUDA tensors with requires_grad) through SplineEAMFunction on
    `system`.  The capture warms up on a side stream, then records the
    forward pass, the adjoint and the loss arithmetic.  Between replays,
    change the parameters in place only (`p.copy_(...)` under torch.no_grad,
    or an optimiser step outside the graph); each replay leaves the loss in
    `self.loss` and the gradients in `self.grads` (the same tensors every
    time, overwritten).  The positions and settings of `system` are part of
    the capture: once a call changes them (`System.epoch` moves on), replay
    raises and the loss must be captured again.
    """

    def __init__(self, system, params, loss_fn, warmup=3):
        self.system = system
        self.params = list(params)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                for p in self.params:
                    p.grad = None
                loss_fn().backward()
        torch.cuda.current_stream().wait_stream(side)
        for p in self.params:
            p.grad = None
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=side):
            loss = loss_fn()
            loss.backward()
        self.loss = loss.detach()
        self.grads = [p.grad for p in self.params]
        self._epoch = system.epoch

    def replay(self):
        """One loss and gradient evaluation on the current stream; returns
        (loss, grads)."""
        if self.system.epoch != self._epoch:
            raise RuntimeError("the system changed since the capture: capture the loss again")
        self.graph.replay()
        # the device now holds the captured coefficients: the next eager
        # upload must not be skipped as unchanged
        self.system._theta = None
        return self.loss, self.grads
