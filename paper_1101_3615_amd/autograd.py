"""F as a differentiable torch operation.

``born(dm, problem)`` returns the Born data ``F dm`` (paper Sec. 1.1: F is the
Frechet derivative of the modelling map at m0; Sec. 2: the linearised wave
equation).  Its backward is the hand-written adjoint sweep ``F*`` (reverse-time
propagation with the zero-lag imaging condition), so the gradient of any loss of
the data is ``F* (dloss/dd)``.  F is linear in dm, so nothing of dm is saved:
the backward reuses the background checkpoints (or g history) that the forward
stored in the context and recomputes the background between checkpoints.
"""
import torch


class BornF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dm, problem):
        ctx.problem = problem
        ctx.dtype = dm.dtype
        return problem.apply_F(dm.detach())

    @staticmethod
    def backward(ctx, grad_d):
        img = ctx.problem.apply_Fadj(grad_d.detach().contiguous())
        return img.to(ctx.dtype), None


def born(dm, problem):
    """Differentiable d = F dm on ``problem`` (a paper_1101_3615_amd.Problem)."""
    return BornF.apply(dm, problem)
