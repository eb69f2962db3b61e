"""Differentiation of the long-range energy and potentials (torch.autograd).

The fast method applies phi = S^T F^-1 C D F S q (eq. matform), with the k-space factor C D real,
even and diagonal, so phi = A(x) q with A symmetric (the self term adds a constant diagonal).
Hence, for E = 1/2 q^T A q (Remark in Sec. 3.1):
    dE/dq_i = phi_i,          dE/dx_i = q_i grad phi_i = -F_i,
which the forward pass already produced: an energy-only loss costs no extra launch. For a loss
that also depends on phi through an upstream gradient g = dL/dphi, one more application with
charges g gives psi = A g and
    dL/dq_i = g_E phi_i + psi_i,
    dL/dx_i = g_E q_i grad phi_i + g_i grad phi_i + q_i grad psi_i,
where the last two terms are the interpolation-side and spreading-side derivatives of
g^T A(x) q. The window gradients are the exact derivatives of the window polynomials, so these
are the exact derivatives of the computed quantities, away from the positions where a support
shifts by one grid point (there the window's edge value psi_0(1)/psi_0(0) ~ eps_w makes the
computed energy jump by that relative amount).
"""
from __future__ import annotations

import torch

from . import BatchPlan, Plan


class _LongRange(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, plan, total=False):
        phi, gphi, E = plan.compute(pos, q, phi=True, grad=True, energy=True, total=total)
        ctx.plan = plan
        ctx.total = total
        ctx.save_for_backward(pos, q, phi, gphi)
        return E, phi

    @staticmethod
    def backward(ctx, gE, gphi_out):
        pos, q, phi, gphi = ctx.saved_tensors
        plan = ctx.plan
        dt = phi.dtype
        ge = gE.to(dt).reshape(()) if gE is not None else torch.zeros((), dtype=dt, device=phi.device)
        dq = ge * phi
        dx = (ge * q)[:, None] * gphi
        if gphi_out is not None and bool(torch.any(gphi_out != 0)):
            g = gphi_out.to(dt).contiguous()
            psi, gpsi, _ = plan.compute(pos, g, phi=True, grad=True, energy=False, total=ctx.total)
            dq = dq + psi
            dx = dx + g[:, None] * gphi + q[:, None] * gpsi
        return (dx if ctx.needs_input_grad[0] else None, dq if ctx.needs_input_grad[1] else None, None, None)


def energy_and_potential(pos: torch.Tensor, q: torch.Tensor, plan: Plan, total: bool = False):
    """Long-range energy E (float64 tensor of shape (1,)) and potentials phi (plan precision),
    differentiable with respect to positions and charges. total=True differentiates the full
    Ewald sum (the real-space residual R is symmetric in the pair too, so the same adjoint
    holds)."""
    return _LongRange.apply(pos, q, plan, total)


def energy(pos: torch.Tensor, q: torch.Tensor, plan: Plan, total: bool = False) -> torch.Tensor:
    """Long-range (or, with total=True, full Ewald) energy, differentiable with respect to
    positions and charges."""
    return _LongRange.apply(pos, q, plan, total)[0]


class _BatchLongRange(torch.autograd.Function):
    """The same adjoint for a batch of independent systems: A is block diagonal (one block per
    system), so the energy gradient of system s reaches only its own particles."""

    @staticmethod
    def forward(ctx, pos, q, plan):
        phi, gphi, E = plan.compute(pos, q, phi=True, grad=True, energy=True)
        ctx.plan = plan
        ctx.save_for_backward(pos, q, phi, gphi)
        return E, phi

    @staticmethod
    def backward(ctx, gE, gphi_out):
        pos, q, phi, gphi = ctx.saved_tensors
        plan = ctx.plan
        dt = phi.dtype
        counts = torch.as_tensor(plan.counts, device=phi.device)
        if gE is None:
            ge = torch.zeros_like(phi)
        else:
            ge = torch.repeat_interleave(gE.to(dt), counts, output_size=phi.shape[0])
        dq = ge * phi
        dx = (ge * q)[:, None] * gphi
        if gphi_out is not None and bool(torch.any(gphi_out != 0)):
            g = gphi_out.to(dt).contiguous()
            psi, gpsi, _ = plan.compute(pos, g, phi=True, grad=True, energy=False)
            dq = dq + psi
            dx = dx + g[:, None] * gphi + q[:, None] * gpsi
        return (dx if ctx.needs_input_grad[0] else None, dq if ctx.needs_input_grad[1] else None, None)


def batch_energy_and_potential(pos: torch.Tensor, q: torch.Tensor, plan: BatchPlan):
    """Energies of every system (float64, shape (nsys,)) and packed potentials, differentiable
    with respect to the packed positions and charges."""
    return _BatchLongRange.apply(pos, q, plan)
