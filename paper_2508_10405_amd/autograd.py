"""Born modelling and migration as a differentiable torch operator.

`BornOp.apply(dm, ctx)` returns the Born data L dm (section 3 of the paper,
L[m0] dm := R du, du from eq. scattereqln); its backward applies the exact
discrete adjoint L^T through the library's migration pass (appendix A:
adjoint-state imaging conditions, section 3 chain rule to lnVp/lnIp).
Nothing that depends on dm is saved for the backward: the migration replays
the background wavefield from the checkpoints the library keeps per model
and acquisition (they do not depend on dm), so memory does not grow with the
number of time steps.  Both directions run in liblsrtm.so; this module only
connects them to autograd.
"""
from __future__ import annotations

import torch

from . import lsrtm


class BornOp(torch.autograd.Function):
    """d = L dm on the context's model and acquisition; backward: L^T."""

    @staticmethod
    def forward(fctx, dm: torch.Tensor, ctx: "lsrtm.Context") -> torch.Tensor:
        fctx.lctx = ctx
        return ctx.born(dm.detach().contiguous())

    @staticmethod
    def backward(fctx, grad_d: torch.Tensor):
        img = fctx.lctx.adjoint(grad_d.detach().contiguous())
        return img, None


def born(dm: torch.Tensor, ctx: "lsrtm.Context") -> torch.Tensor:
    return BornOp.apply(dm, ctx)


def misfit(dm: torch.Tensor, ctx: "lsrtm.Context", d_obs: torch.Tensor) -> torch.Tensor:
    """0.5 ||L dm - d_obs||^2 (section 3, J(dm)) as a differentiable scalar."""
    r = born(dm, ctx) - d_obs
    return 0.5 * torch.dot(r, r)
