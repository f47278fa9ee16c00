"""torch.autograd.Function over the NEP library: energy and forces as differentiable
outputs of the network parameters theta = (W0, b0, w1, b1) and of the positions.

Forward runs the library's descriptor, network and force kernels
(``nep_train_forward``); backward runs its weight-gradient kernel
(``nep_train_backward``: descriptor JVP along dL/dF, network double backward and an
MFMA reduction over atoms) and returns dL/dx = -dL/dE * F for the positions (the
force kernel is the energy's position backward). Second derivatives with respect
to positions (a force-dependent loss differentiated by positions) are not provided.
"""
from __future__ import annotations

from typing import Optional

import torch

from .nep import NEPSystem


class NEPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: Optional[torch.Tensor], theta: torch.Tensor, system: NEPSystem, slot: int = 0,
                skin: float = 1.0):
        if x is not None:
            system.set_positions(x.detach())
            system.build_neighbors(skin)
        E, F = system.train_forward(slot, theta)
        ctx.set_materialize_grads(False)
        ctx.system, ctx.slot, ctx.skin = system, slot, skin
        ctx.generation = system.generation
        ctx.save_for_backward(x.detach() if x is not None else None, theta.detach(), F)
        ctx.has_x = x is not None
        return torch.tensor(E, dtype=torch.float64, device=F.device), F

    @staticmethod
    def backward(ctx, gE, gF):
        x, theta, F = ctx.saved_tensors
        s = ctx.system
        if s.generation != ctx.generation:
            # the system was used for something else since forward: restore this frame
            if x is None:
                raise RuntimeError("system state changed since forward and no positions were given")
            s.set_positions(x)
            s.build_neighbors(ctx.skin)
            s.train_forward(ctx.slot, theta)
        ge = float(gE) if gE is not None else 0.0
        grad_theta = None
        if ctx.needs_input_grad[1]:
            grad_theta = s.train_backward(ctx.slot, theta, ge, gF)
        grad_x = None
        if ctx.has_x and ctx.needs_input_grad[0]:
            if gF is not None and bool(torch.any(gF != 0)):
                raise NotImplementedError("second derivatives with respect to positions are not provided")
            grad_x = (-ge) * F.to(torch.float64)
        return grad_x, grad_theta, None, None, None


def energy_forces(system: NEPSystem, theta: torch.Tensor, x: Optional[torch.Tensor] = None, slot: int = 0,
                  skin: float = 1.0):
    """(E, F) with autograd support for theta (and, for the energy, x)."""
    return NEPFunction.apply(x, theta, system, slot, skin)


def energy_force_loss(systems_frames, theta, labels, slot=0, lam_e=1.0, lam_f=1.0, skin=1.0):
    """Mean over frames of lam_e (dE/N)^2 + lam_f sum|dF|^2 / (3N).

    systems_frames: list of (system, x tensor or None); labels: list of (E_ref, F_ref tensor).
    """
    total = 0.0
    for (s, x), (e_ref, f_ref) in zip(systems_frames, labels):
        E, F = energy_forces(s, theta, x, slot, skin)
        n = F.shape[0]
        de = (E - e_ref) / n
        df = F.to(torch.float64) - f_ref.to(torch.float64)
        total = total + lam_e * de * de + lam_f * (df * df).sum() / (3 * n)
    return total / len(systems_frames)
