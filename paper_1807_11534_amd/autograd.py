"""torch.autograd wrappers around the HIP forward and adjoint kernels.

FitTerm:  f = (z - c1)^2 - (z - c2)^2 + gamma P        (Sec. 1, eq. CV / eq. DS)
RDSolve:  u = restricted dual iteration of f (Sec. 2.1, Sec. 3), unrolled for
          `iters` iterations from u0 = H(-f), p0 = 0; the restricted domain and
          u0 are held fixed under differentiation.

Both functions only move pointers: forward and backward run in librdseg.so.
Scalar parameters (c1, c2, gamma, lambda) are CPU tensors (or Python floats)
so their values can be passed by value through the C ABI; their gradients are
returned on the CPU in the parameter's dtype.
"""
import math

import torch

from . import rdseg


def _val(x):
    return float(x.item()) if isinstance(x, torch.Tensor) else float(x)


def _grad_like(g, x):
    if not isinstance(x, torch.Tensor):
        return None
    return g.detach().cpu().to(x.dtype).reshape(x.shape)


class FitTerm(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, c1, c2, gamma, P=None):
        f = rdseg.fit_forward(z, _val(c1), _val(c2), _val(gamma), P)
        if P is not None:
            ctx.save_for_backward(z, P)
        else:
            ctx.save_for_backward(z)
        ctx.has_P = P is not None
        ctx.c = (_val(c1), _val(c2))
        ctx.params = (c1, c2, gamma)
        return f

    @staticmethod
    def backward(ctx, grad_f):
        saved = ctx.saved_tensors
        z = saved[0]
        P = saved[1] if ctx.has_P else None
        a, b, g = rdseg.fit_backward(z, ctx.c[0], ctx.c[1], rdseg.as_grid_of(grad_f, z), P)
        c1, c2, gamma = ctx.params
        return None, _grad_like(a, c1), _grad_like(b, c2), _grad_like(g, gamma), None


class RDSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, lam, theta=rdseg.THETA, tau=rdseg.TAU, delta=math.inf, iters=100,
                ckpt_every=30, tile=(32, 32), iters_per_launch=2):
        lamv = _val(lam)
        u, v, p, tape = rdseg.solve(f, lamv, theta, tau, delta, iters, tile=tile,
                                    iters_per_launch=iters_per_launch, ckpt_every=ckpt_every)
        ctx.save_for_backward(f, tape)
        ctx.args = (lamv, theta, tau, delta, iters, ckpt_every)
        ctx.lam = lam
        return u

    @staticmethod
    def backward(ctx, grad_u):
        f, tape = ctx.saved_tensors
        lamv, theta, tau, delta, iters, ckpt_every = ctx.args
        gf, gl = rdseg.backward(f, lamv, theta, tau, delta, iters, ckpt_every, tape,
                                rdseg.as_grid_of(grad_u, f))
        return gf, _grad_like(gl, ctx.lam), None, None, None, None, None, None, None
