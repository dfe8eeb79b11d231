"""render_residuals as a torch.autograd.Function.

forward:  r = H(x) - C per ray (Eq. 3-6), shape [rays, 3] (plus the opacity residual of Eq. 10
          as a fourth column when the scene has it on), from the library's render pass.
backward: dl/dx = J^T (dl/dr), from the library's adjoint pass, which re-marches every ray
          instead of keeping per-sample state from the forward pass.
"""
from __future__ import annotations

import torch


class RenderResiduals(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, scene) -> torch.Tensor:
        r, _ = scene.render_residuals(x.detach().contiguous())
        ctx.scene = scene
        ctx.save_for_backward(x)
        return r.view(-1, scene.n_res)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (x,) = ctx.saved_tensors
        y = ctx.scene.apply_Jt(x.detach().contiguous(), g.detach().contiguous().view(-1).to(torch.float32))
        return y, None


def render_residuals(x: torch.Tensor, scene) -> torch.Tensor:
    return RenderResiduals.apply(x, scene)
