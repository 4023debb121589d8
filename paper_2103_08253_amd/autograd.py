"""torch.autograd.Function wrappers around the hand-written backward kernels.

* DmnLinear: Cbar = DMN^L(C1, C2; w, n) with the laminate-tree VJP
  (dmn_homogenize_backward) as its backward.
* DmnPathStress: final effective stresses of a load path, with the load-step
  adjoint swept over checkpointed segments as its backward (gradients w.r.t.
  the leaf weights and normals).

Normals are taken as passed.  `normals_from_angles` is a convenience for
callers who compose the map with their own torch code (torch then
differentiates the angle map); the library's training step
(`training.TrainingStepGraph`) does not use it: there the angle chain and the
optimiser run in the update kernel.
"""
import torch

from .api import dmn_homogenize_backward, dmn_homogenize_linear
from .path import adjoint_sweep, forward_checkpointed


def normals_from_angles(alpha: torch.Tensor, beta: torch.Tensor) -> torch.Tensor:
    """n = (sin a cos b, sin a sin b, cos a) (spherical parameterisation)."""
    return torch.stack([torch.sin(alpha) * torch.cos(beta), torch.sin(alpha) * torch.sin(beta),
                        torch.cos(alpha)], dim=-1).contiguous()


class DmnLinear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, n, C1, C2):
        w, n, C1, C2 = (t.contiguous() for t in (w, n, C1, C2))
        Cbar, _ = dmn_homogenize_linear(w, n, C1, C2)
        ctx.save_for_backward(w, n, C1, C2)
        return Cbar

    @staticmethod
    def backward(ctx, gCbar):
        w, n, C1, C2 = ctx.saved_tensors
        want = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
        gw, gn, gC1, gC2, _ = dmn_homogenize_backward(w, n, C1, C2, gCbar.contiguous(),
                                                      want_input_grads=want)
        return gw, gn, gC1, gC2


class DmnPathStress(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, n, E_path, fiber, matrix, checkpoint_every=10):
        w, n, E_path = w.contiguous(), n.contiguous(), E_path.contiguous()
        sigma, cks = forward_checkpointed(w, n, E_path, fiber, matrix, checkpoint_every)
        ctx.save_for_backward(w, n, E_path)
        ctx.checkpoints = cks
        ctx.cfg = (fiber, matrix, checkpoint_every)
        return sigma

    @staticmethod
    def backward(ctx, g_sigma):
        w, n, E_path = ctx.saved_tensors
        fiber, matrix, ck = ctx.cfg
        gw, gn = adjoint_sweep(w, n, E_path, ctx.checkpoints, g_sigma.contiguous(), fiber,
                               matrix, ck)
        return gw, gn, None, None, None, None


def dmn_linear(w, n, C1, C2):
    return DmnLinear.apply(w, n, C1, C2)


def dmn_path_stress(w, n, E_path, fiber, matrix, checkpoint_every=10):
    return DmnPathStress.apply(w, n, E_path, fiber, matrix, checkpoint_every)
