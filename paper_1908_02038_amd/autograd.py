"""torch.autograd wrappers over the library's kernels.

``energy(ctx, pos, box, pot)`` returns E(x) as a differentiable scalar:

* ``EnergyFn``: forward runs the force pass for E; its backward is the force
  kernel itself, since dE/dx = -F (Sec. 2.1 defines F as -grad E).
* ``ForceFn``: F(x) = -grad E, the force kernel; its backward is the
  Hessian-vector-product kernel (dF/dx = -H, H symmetric, so the
  vector-Jacobian product with g is -H g).

So ``torch.autograd.grad(E, x, create_graph=True)`` yields -F from the force
kernel, and differentiating that again applies the HVP kernel: first and
second derivatives both come from the hand-written kernels, none from
autograd tracing.  Positions are (n, 3) float64 CUDA tensors in the caller's
order; every call works on the current torch stream.
"""
from __future__ import annotations

import torch


class ForceFn(torch.autograd.Function):
    """F(x) from the force kernel; backward g -> -H g from the HVP kernel."""

    @staticmethod
    def forward(ctx, pos, fctx, box, pot):
        _, f = fctx.fire_energy_forces_dev(pos.detach().contiguous(), box, pot)
        ctx.save_for_backward(pos)
        ctx.fctx, ctx.box, ctx.pot = fctx, box, pot
        return f

    @staticmethod
    def backward(ctx, grad_f):
        (pos,) = ctx.saved_tensors
        hu = ctx.fctx.fire_hvp_dev(pos.detach().contiguous(), grad_f.detach().contiguous(), ctx.box, ctx.pot)
        return -hu, None, None, None


class EnergyFn(torch.autograd.Function):
    """E(x); backward grad_E -> -grad_E * F(x) with F from ForceFn, so that a
    graph built for double backward reaches the HVP kernel."""

    @staticmethod
    def forward(ctx, pos, fctx, box, pot):
        e, _ = fctx.fire_energy_forces_dev(pos.detach().contiguous(), box, pot)
        ctx.save_for_backward(pos)
        ctx.fctx, ctx.box, ctx.pot = fctx, box, pot
        return e.reshape(())

    @staticmethod
    def backward(ctx, grad_e):
        (pos,) = ctx.saved_tensors
        f = ForceFn.apply(pos, ctx.fctx, ctx.box, ctx.pot)
        return -grad_e * f, None, None, None


def energy(fctx, pos: torch.Tensor, box, pot) -> torch.Tensor:
    """Differentiable E(x) for an (n, 3) float64 CUDA tensor on context fctx."""
    if not (pos.is_cuda and pos.dtype == torch.float64 and pos.dim() == 2 and pos.shape[1] == 3):
        raise TypeError("pos must be an (n, 3) float64 CUDA tensor")
    return EnergyFn.apply(pos, fctx, box, pot)


def forces(fctx, pos: torch.Tensor, box, pot) -> torch.Tensor:
    """Differentiable F(x) = -grad E (its backward is the HVP kernel)."""
    if not (pos.is_cuda and pos.dtype == torch.float64 and pos.dim() == 2 and pos.shape[1] == 3):
        raise TypeError("pos must be an (n, 3) float64 CUDA tensor")
    return ForceFn.apply(pos, fctx, box, pot)
