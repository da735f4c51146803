"""Differentiable CVP operators.

Project.apply(x, geom, opts) = A x; its backward is the hand-written
backprojector A^T (the exact adjoint of the same weights, Sec. III-D), and
BackProject.apply(b, geom, opts) = A^T b has the projector as its backward.
"""
import torch

from . import cvp


class Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, geom, opts=cvp.Options()):
        ctx.geom, ctx.opts = geom, opts
        return cvp.project(x.contiguous(), geom, opts)

    @staticmethod
    def backward(ctx, grad_b):
        grad_x = cvp.backproject(grad_b.contiguous(), ctx.geom, ctx.opts) if ctx.needs_input_grad[0] else None
        return grad_x, None, None


class BackProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, geom, opts=cvp.Options()):
        ctx.geom, ctx.opts = geom, opts
        return cvp.backproject(b.contiguous(), geom, opts)

    @staticmethod
    def backward(ctx, grad_x):
        grad_b = cvp.project(grad_x.contiguous(), ctx.geom, ctx.opts) if ctx.needs_input_grad[0] else None
        return grad_b, None, None


def project(x, geom, opts=cvp.Options()):
    return Project.apply(x, geom, opts)


def backproject(b, geom, opts=cvp.Options()):
    return BackProject.apply(b, geom, opts)
