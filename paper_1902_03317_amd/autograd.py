"""Differentiable CP model at the nonzeros (torch.autograd.Function).

* :class:`CPSample` -- forward samples the rank-R CP model at every nonzero,
  mhat_m = sum_r prod_k U_k[i_k(m), r]; backward gives each factor the
  MTTKRP of the tensor's pattern with the incoming gradient as values.
* :func:`cp_loss` -- the observed-entry least-squares loss
  1/2 sum_m (mhat_m - x_m)^2 of a gradient-based CP fit. The default fused
  form computes the loss and every factor's gradient (the residual-weighted
  MTTKRP) in one pass per mode during forward, recomputing the residual in
  each mode's order instead of storing it; backward only scales the stored
  gradients by the upstream derivative. ``fused=False`` stores the residual
  in forward and runs the residual-weighted MTTKRP in backward.
  ``shadows`` (bf16 copies of the fp32 ``masters``) makes the products read
  bf16 factors while gradients flow to the fp32 masters.
All arithmetic runs in libpasta's HIP kernels.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import api
from ._lib import check, lib


def _scale_(t: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    """t *= s in place, s a device scalar (fp64), via the library's scale kernel."""
    s = s.detach().to(torch.float64).reshape(()).contiguous()
    check(lib.pasta_scale_f32(t.data_ptr(), t.numel(), s.data_ptr(), api._stream()), "pasta_scale_f32")
    return t


class CPSample(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X: api.Coo, *factors):
        ctx.X = X
        ctx.save_for_backward(*factors)
        return api.cp_sample(X, [f.detach() for f in factors])

    @staticmethod
    def backward(ctx, g):
        factors = [f.detach() for f in ctx.saved_tensors]
        g = g.detach().to(torch.float32).contiguous()
        grads = []
        for n in range(len(factors)):
            if ctx.needs_input_grad[n + 1]:
                grads.append(api.mttkrp(ctx.X, factors, n, vals=g))
            else:
                grads.append(None)
        return (None, *grads)


class _CPLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X: api.Coo, shadows, fused: bool, *masters):
        facs = [f.detach() for f in (shadows if shadows is not None else masters)]
        ctx.X = X
        ctx.fused = fused
        if fused:
            loss, grads = api.cp_grad(X, facs)
            ctx.save_for_backward(*grads)
        else:
            resid, loss = api.cp_residual_loss(X, facs)
            ctx.facs = facs
            ctx.save_for_backward(resid)
        return loss

    @staticmethod
    def backward(ctx, gl):
        if ctx.fused:
            grads = [_scale_(g.clone(), gl) for g in ctx.saved_tensors]
        else:
            (resid,) = ctx.saved_tensors
            grads = [_scale_(api.mttkrp(ctx.X, ctx.facs, n, vals=resid), gl) for n in range(len(ctx.facs))]
        return (None, None, None, *grads)


def cp_loss(X: api.Coo, masters: Sequence[torch.Tensor], shadows: Optional[Sequence[torch.Tensor]] = None,
            fused: bool = True) -> torch.Tensor:
    """1/2 sum over nonzeros of (CP model - value)^2 as a differentiable fp64 scalar."""
    return _CPLoss.apply(X, None if shadows is None else list(shadows), fused, *masters)


CPLoss = _CPLoss


def adam_step(params, grads, exp_avg, exp_avg_sq, step: int, lr: float = 1e-2, betas=(0.9, 0.999),
              eps: float = 1e-8, shadows=None):
    """One fused Adam update of fp32 factors; refreshes bf16 shadows in the same pass."""
    for i, (p, g, m, v) in enumerate(zip(params, grads, exp_avg, exp_avg_sq)):
        sh = None if shadows is None else shadows[i]
        check(lib.pasta_adam_step(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                                  None if sh is None else sh.data_ptr(), p.numel(), float(lr), float(betas[0]),
                                  float(betas[1]), float(eps), int(step), api._stream()), "pasta_adam_step")
