"""torch.autograd wrapper of the sampled core update and its hand-written adjoint.

``sketched_core_update(X, factors, lam, samples, ...)`` returns the core g of
the sampled ridge update (Alg. 3 with Alg. 1) and records a node whose
backward calls ``tucker_core_update_sketched_adjoint`` with the same sample
set: gradients flow to the factor matrices and to the tensor entries (nonzero
only at sampled observed entries).  The sample set is a constant of the
gradient -- the leverage-score weights are not differentiated.
"""
import torch

from . import tucker


class SketchedCoreUpdate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, lam, samples, seed, counter, precision, mask, idx, weight, refine_max,
                *factors):
        F = [A.detach() for A in factors]
        G, idx_u, w_u = tucker.core_update_sketched(
            X.detach(), F, lam, samples, seed=seed, counter=counter, precision=precision, mask=mask,
            idx=idx, weight=weight, refine_max=refine_max, return_samples=True)
        ctx.save_for_backward(X.detach(), G, idx_u, w_u, *F)
        ctx.cfg = (lam, precision, mask, refine_max)
        ctx.mark_non_differentiable(idx_u, w_u)
        return G, idx_u, w_u

    @staticmethod
    def backward(ctx, gbar, _idx_bar, _w_bar):
        X, G, idx, w, *F = ctx.saved_tensors
        lam, precision, mask, refine_max = ctx.cfg
        want_x = ctx.needs_input_grad[0]
        fbar, xbar = tucker.core_update_sketched_adjoint(
            X, F, lam, idx, w, G, gbar.contiguous(), precision=precision, mask=mask,
            refine_max=refine_max, want_x=want_x)
        grads = [xbar if want_x else None] + [None] * 9
        grads += [fb if need else None for fb, need in zip(fbar, ctx.needs_input_grad[10:])]
        return tuple(grads)


def sketched_core_update(X, factors, lam, samples, seed=0, counter=0, precision="f64", mask=None,
                         idx=None, weight=None, refine_max=20, return_samples=False):
    """Differentiable sampled core update; optionally also returns the samples used."""
    G, idx_u, w_u = SketchedCoreUpdate.apply(X, float(lam), samples, seed, counter, precision, mask,
                                             idx, weight, refine_max, *factors)
    if return_samples:
        return G, idx_u, w_u
    return G
