"""CPU emulation of the BF16 training path's rounding points, the ground for
the tolerance of its gradient tests.

The policy network (Sec. VI-A) runs forward in float64 with the values the
BF16 path stores in BF16 rounded to BF16 (round to nearest even): the
activations of layers 1..5 and the weights of layers 2..5 (layers 1 and 6
keep FP32 weights). The weight gradient of sum(g_prob * p) then follows by
automatic differentiation through those rounded values, the rounding
passing gradients through unchanged, as the BF16 backward uses the rounded
activations and weights. The BF16 path also rounds its gradient maps, which
this leaves out (about 3e-6 of relative error on the gradient). With
rounding off it is the exact gradient, which a CPU test pins to the
oracle's."""
import numpy as np
import torch
import torch.nn.functional as F

CH = (2, 32, 32, 32, 32, 32, 1)


class _RoundBF16(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return x.to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


def weight_gradient(w, c, z, g_prob, bf16=True):
    """d/dw of sum(g_prob * sigmoid(x)) for the flat weights w (per layer the
    OIHW 3x3 weights, then the biases), contone c and noise z [B, H, W];
    with bf16 the path's rounding points, else exact float64. Returns the
    gradient and the probabilities."""
    rnd = _RoundBF16.apply if bf16 else (lambda t: t)
    wt = torch.tensor(np.asarray(w, dtype=np.float64), requires_grad=True)
    a = torch.stack([torch.as_tensor(np.asarray(c, dtype=np.float64)),
                     torch.as_tensor(np.asarray(z, dtype=np.float64))], dim=1)
    off = 0
    nl = len(CH) - 1
    for k in range(nl):
        ci, co = CH[k], CH[k + 1]
        n = co * ci * 9
        wk = wt[off:off + n].view(co, ci, 3, 3)
        bk = wt[off + n:off + n + co]
        off += n + co
        if 1 <= k <= 4:
            wk = rnd(wk)
        a = F.conv2d(a, wk, bk, padding=1)
        if k < nl - 1:
            a = rnd(torch.relu(a))
    p = torch.sigmoid(a[:, 0])
    (p * torch.as_tensor(np.asarray(g_prob, dtype=np.float64))).sum().backward()
    return wt.grad.numpy(), p.detach().numpy()


def layer_slices():
    """(lo, hi) of each layer's weights and bias in the flat vector."""
    out, off = [], 0
    for k in range(len(CH) - 1):
        n = CH[k + 1] * CH[k] * 9 + CH[k + 1]
        out.append((off, off + n))
        off += n
    return out
