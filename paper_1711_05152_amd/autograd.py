"""Differentiable multiple rank-1 lattice transforms (torch.autograd.Function).

For a complex-linear map out = B x, PyTorch's convention for complex gradients makes the
backward pass apply the adjoint B^H to the incoming gradient, so each Function's backward is the
library's transform in the other direction:

  Mr1lFFT        c = F y   (Alg. 2, weights "paper")     backward: F^H g (scatter + inverse DFTs)
  Mr1lFFTAdj     y = F^H c                                backward: F g
  Mr1lSynth      y = A c   (Fourier matrix, "eval")      backward: A^H g
  Mr1lAnalysis   c = A^H y                                backward: A g

and the fused sample-domain least-squares loss of a fit y ~ A c on the plan's lattices,

  WeightedLsq    loss = 1/2 sum_l (1/M_l) ||s_l - y_l||^2  backward: g (1/M_l)(s_l - y_l)

(one pass over s and y in the library each way, instead of the elementwise operations of an
autograd graph over the whole sample vector).

Plans carry the direction-independent data (frequencies, lattices, filter spectra); the
weights of the plan select F or A.
"""
from __future__ import annotations

import torch

__all__ = ["Mr1lFFT", "Mr1lFFTAdj", "Mr1lSynth", "Mr1lAnalysis", "WeightedLsq", "mr1l_fft", "mr1l_synth"]


def _need(plan, weights):
    if plan.weights != weights:
        raise ValueError(f"this Function needs a plan with weights={weights!r}")


class Mr1lFFT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, samples, plan):
        _need(plan, "paper")
        ctx.plan = plan
        return plan.forward(samples)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.adjoint(g.contiguous()), None


class Mr1lFFTAdj(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeffs, plan):
        _need(plan, "paper")
        ctx.plan = plan
        return plan.adjoint(coeffs)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.forward(g.contiguous()), None


class Mr1lSynth(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeffs, plan):
        _need(plan, "eval")
        ctx.plan = plan
        return plan.adjoint(coeffs)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.forward(g.contiguous()), None


class Mr1lAnalysis(torch.autograd.Function):
    @staticmethod
    def forward(ctx, samples, plan):
        _need(plan, "eval")
        ctx.plan = plan
        return plan.forward(samples)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.adjoint(g.contiguous()), None


class WeightedLsq(torch.autograd.Function):
    """Real float64 loss of samples s [n_rhs, sum M] against data y (y is not differentiated)."""

    @staticmethod
    def forward(ctx, s, y, plan):
        loss = torch.empty((), dtype=torch.float64, device=s.device)
        plan.lsq_residual(s, y, loss=loss)
        ctx.save_for_backward(s, y)
        ctx.plan = plan
        return loss

    @staticmethod
    def backward(ctx, g):
        s, y = ctx.saved_tensors
        grad = torch.empty_like(s)
        ctx.plan.lsq_residual(s, y, grad=grad, scale=g.detach().to(torch.float64).reshape(()).contiguous())
        return grad, None, None


def mr1l_fft(samples, plan):
    return Mr1lFFT.apply(samples, plan)


def mr1l_synth(coeffs, plan):
    return Mr1lSynth.apply(coeffs, plan)
