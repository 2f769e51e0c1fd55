"""Gradient of a bead-velocity loss with respect to the fluid's shear and bulk
relaxation rates and the bead friction, as a torch.autograd.Function.

The forward runs a window of LB steps on the GPU (C ABI lb_window_forward)
and returns the bead velocities after every step; the backward hands
dJ/dv to the library's hand-written adjoint (lb_window_backward), which
returns dJ/d(omega_shear, omega_bulk, zeta) per box.  The loss itself is any
torch function of the velocities; vacf() and vacf_loss() give the bead
velocity autocorrelation and its normalised squared mismatch to a target.
"""
from __future__ import annotations

import torch


class LBWindow(torch.autograd.Function):
    """theta [n_boxes, 3] float64 = (omega_shear, omega_bulk, zeta) per box ->
    bead velocities [T, sum N, 3] after each of T steps (float64, CPU)."""

    @staticmethod
    def forward(ctx, theta, system, T: int, k: int):
        th = theta.detach().cpu().double()
        for b in range(th.shape[0]):
            system.set_rates(b, *th[b].tolist())
        vh = system.window_forward(T, k)
        ctx.system = system
        return torch.from_numpy(vh.copy())

    @staticmethod
    def backward(ctx, g):
        grad = ctx.system.window_backward(g.detach().cpu().double().numpy())
        return torch.from_numpy(grad), None, None, None


def vacf(vh: torch.Tensor, tmax: int) -> torch.Tensor:
    """C(tau) = (1/N) (1/(T - tau)) sum_t0 sum_b v_b(t0) . v_b(t0 + tau), tau = 0..tmax."""
    T, N = vh.shape[0], vh.shape[1]
    out = []
    for tau in range(tmax + 1):
        out.append((vh[: T - tau] * vh[tau:]).sum() / (N * (T - tau)))
    return torch.stack(out)


def vacf_loss(vh: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """sum_tau (C(tau) - C*(tau))^2 / C*(0)^2."""
    c = vacf(vh, target.shape[0] - 1)
    return ((c - target) ** 2).sum() / target[0] ** 2
