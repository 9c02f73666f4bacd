"""torch.autograd wrappers over the hand-written forward and backward kernels.

PolicyConv: probs = sigmoid(CNN(c, z; theta)) with the conv stack's own
backward (input gradients and weight gradients in HIP).
HalftoneLoss: the training loss whose gradient is the Local Expectation
estimator for the main batch (dL_MARL/dp = -dR/B) plus w_a times the
anisotropy-suppressing loss for the gray batch. Its forward value is the
scalar -mean(R) + w_a L_AS that the library returns (the reported
surrogate); its backward is the estimator, not the derivative of that value
with respect to p.
"""
import torch

from . import binding as hb


class PolicyConv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, contone, seeds, step, noise_kind, precision):
        probs, ws = hb.halftone_policy_forward(weights, contone, seeds, step, noise_kind,
                                               precision)
        ctx.save_for_backward(weights, probs)
        ctx.ws = ws
        ctx.precision = precision
        return probs

    @staticmethod
    def backward(ctx, grad_probs):
        weights, probs = ctx.saved_tensors
        gw = hb.halftone_policy_backward(weights, grad_probs.contiguous(), probs, ctx.ws,
                                         ctx.precision)
        return gw, None, None, None, None, None


class HalftoneLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, probs, actions, contone, probs_gray, prm):
        out = hb.halftone_loss(actions, contone, probs_gray, prm)
        B = contone.shape[0]
        ctx.save_for_backward(probs, actions, contone, probs_gray)
        ctx.prm = prm
        return out[3 * B + 1]

    @staticmethod
    def backward(ctx, g):
        probs, actions, contone, probs_gray = ctx.saved_tensors
        gp, gg = hb.halftone_loss_backward(actions, contone, probs, probs_gray, ctx.prm,
                                           hb.HS_WRT_PROB)
        return gp * g, None, None, (gg * g if gg is not None else None), None


def policy(weights, contone, seeds, step=0, noise_kind=hb.HS_NOISE_GAUSS, precision=hb.HS_FP32):
    return PolicyConv.apply(weights, contone, seeds, step, noise_kind, precision)


def halftone_loss(probs, actions, contone, probs_gray=None, prm=None):
    return HalftoneLoss.apply(probs, actions, contone, probs_gray,
                              prm or hb.default_loss_params())
