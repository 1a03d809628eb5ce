"""torch.autograd.Function wrappers and the two host drivers built on them:
mean shift (a density-gradient application, Sec. 1) and bandwidth bisection
(Sec. 5, "Bandwidth selection").
"""
from __future__ import annotations

import math

import torch

from . import api


def _h_value(h) -> float:
    return float(h.detach().cpu()) if isinstance(h, torch.Tensor) else float(h)


class ExactKDE(torch.autograd.Function):
    """out = exact KDE of Y against X; differentiable in Y and h (FP32 operands).
    `prepared`: an FP32 prepared set of X (api.prepare), used by both passes."""

    @staticmethod
    def forward(ctx, Y, h, X, kernel="gaussian", prepared=None):
        hv = _h_value(h)
        out = api.kde_exact(X, Y.detach().contiguous(), hv, kernel, "fp32", prepared=prepared)
        ctx.save_for_backward(X, Y)
        ctx.hv, ctx.kernel, ctx.prepared = hv, kernel, prepared
        ctx.h_is_tensor = isinstance(h, torch.Tensor)
        ctx.h_device = h.device if ctx.h_is_tensor else None
        return out

    @staticmethod
    def backward(ctx, grad_out):
        X, Y = ctx.saved_tensors
        need_y, need_h = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gy, gh = api.kde_exact_backward(X, Y.detach().contiguous(), ctx.hv, grad_out, ctx.kernel,
                                        need_y, need_h and ctx.h_is_tensor,
                                        prepared=ctx.prepared)
        gh_out = gh.reshape(()).to(ctx.h_device) if gh is not None else None
        return gy, gh_out, None, None, None


class DeannKDE(torch.autograd.Function):
    """out = DEANN estimate; the index sets are saved for the backward."""

    @staticmethod
    def forward(ctx, Y, h, X, k, m, kernel="gaussian", seed=0, query_offset=0, word2=0,
                precision="fp32", start=None, index=None, prepared=None):
        hv = _h_value(h)
        if start is None:   # draws with repetition (Algorithm 1)
            out, nn, sm = api.deann_query(X, Y.detach().contiguous(), hv, k, m, kernel, seed,
                                          query_offset, word2, precision, prepared=prepared)
        else:               # permuted random sampling from running index `start`
            out, nn, sm = api.deann_query_permuted(X, Y.detach().contiguous(), hv, k, m, kernel,
                                                   seed, start, precision, index=index)
        ctx.save_for_backward(X, Y, nn, sm)
        ctx.hv, ctx.kernel, ctx.k, ctx.m = hv, kernel, k, m
        ctx.h_is_tensor = isinstance(h, torch.Tensor)
        ctx.h_device = h.device if ctx.h_is_tensor else None
        ctx.mark_non_differentiable(nn, sm)
        return out, nn, sm

    @staticmethod
    def backward(ctx, grad_out, _gnn=None, _gsm=None):
        X, Y, nn, sm = ctx.saved_tensors
        need_y, need_h = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gy, gh = api.deann_query_backward(X, Y.detach().contiguous(), ctx.hv, ctx.k, ctx.m, nn, sm,
                                          grad_out, ctx.kernel, need_y, need_h and ctx.h_is_tensor)
        gh_out = gh.reshape(()).to(ctx.h_device) if gh is not None else None
        return (gy, gh_out) + (None,) * 11


def exact_kde(Y, h, X, kernel="gaussian", prepared=None):
    """Exact KDE with autograd; `prepared`: an FP32 prepared set of X."""
    return ExactKDE.apply(Y, h, X, kernel, prepared)


def deann_kde(Y, h, X, k, m, kernel="gaussian", seed=0, query_offset=0, word2=0,
              precision="fp32", start=None, index=None, prepared=None):
    """DEANN estimate with autograd; start (not None) selects permuted random
    sampling from that running index instead of draws with repetition, with
    the rows of a PermutedIndex when one is given; `prepared`: a prepared set
    of X in `precision` (draws with repetition only)."""
    out, _, _ = DeannKDE.apply(Y, h, X, k, m, kernel, seed, query_offset, word2, precision, start,
                               index, prepared)
    return out


def mean_shift(X, Y, h, steps, method="exact", k=0, m=0, seed=0, precision="fp32"):
    """Gaussian mean shift y <- y + h^2 grad(mu)/mu, i.e. the kernel-weighted mean
    of the rows (with DEANN weights for method="deann").  Exact: density and
    gradient from one pass (kde_exact_with_grad).  DEANN: the estimate and its
    gradient from one gather (deann_query_with_grad); step t draws with counter
    word 2 = t.  X is prepared once for all steps (deann_prepare).  Returns the
    float32 end point [q, d]."""
    Y = Y.detach().clone().contiguous()
    pre = api.prepare(X, "fp32" if method == "exact" else precision) if steps > 0 else None
    for t in range(steps):
        if method == "exact":
            mu, g, _ = api.kde_exact_with_grad(X, Y, float(h), "gaussian", True, False,
                                               prepared=pre)
        else:
            mu, g, _, _, _ = api.deann_query_with_grad(X, Y, float(h), k, m, "gaussian", seed, 0, t,
                                                       precision, need_grad_h=False,
                                                       return_indices=False, prepared=pre)
        api.mean_shift_update(Y, g, mu, float(h), out=Y)
    return Y


def bisect_h(X, Y, target: float, kernel="gaussian", stat="mean", rel_tol=0.01,
             lo=-20.0, hi=20.0, max_iter=200) -> float:
    """Bandwidth whose mean (or median) exact KDE over Y is within rel_tol of target,
    by bisection on log h with the FP32 exact path (X prepared once)."""
    pre = api.prepare(X, "fp32")
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        h = math.exp(mid)
        v = api.kde_exact(X, Y, h, kernel, "fp32", prepared=pre)
        val = float(v.mean() if stat == "mean" else v.median())
        if abs(val - target) <= rel_tol * target:
            return h
        if val < target:
            lo = mid
        else:
            hi = mid
    raise RuntimeError("bisection did not converge")
