"""FP64 reference of the warm-start network (test infrastructure only).

A plain multilayer perceptron: x -> tanh(W1 x + b1) -> tanh(W2 . + b2) ->
tanh(W3 . + b3) -> W4 . + b4, mean-squared error against targets.  The GPU
keeps the weights in BF16 and accumulates in FP32; the reference takes the
same (BF16-rounded) weights as FP64 and computes the loss and all gradients
in FP64 by the chain rule, so the GPU gradients can be checked against it.
This part is not from the paper: it is the learned warm start of the solve.
"""
import numpy as np


def bf16_round(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, X):
    """params: list of (W, b) with W (out, in); returns list of layer outputs."""
    acts = [X]
    h = X
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        h = np.tanh(z) if li < len(params) - 1 else z
        acts.append(h)
    return acts


def loss_and_grads(params, X, T):
    """Mean over the batch of the summed squared error, and its gradients."""
    acts = forward(params, X)
    B = X.shape[0]
    Y = acts[-1]
    loss = np.sum((Y - T) ** 2) / B
    dh = 2.0 * (Y - T) / B
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        dz = dh if li == len(params) - 1 else dh * (1.0 - acts[li + 1] ** 2)
        grads[li] = (dz.T @ acts[li], dz.sum(axis=0))
        dh = dz @ W
    return loss, grads
