"""Pins of the warm-start network's FP64 reference (oracle/mlp.py): BF16
rounding against torch's conversion and hand-made ties, gradients against
central differences and against torch autograd in FP64."""
import numpy as np
import pytest
import torch

import oracle.mlp as M
from inputs import SEED, mlp_case, uniforms


def _unpack(dims, flat):
    out, k = [], 0
    flat = np.asarray(flat, dtype=np.float64)
    for o, i in dims:
        W = flat[k:k + o * i].reshape(o, i)
        k += o * i
        b = flat[k:k + o]
        k += o
        out.append((W, b))
    return out


def test_bf16_round_matches_torch_conversion():
    u = np.array(uniforms(SEED + 7, 4000))
    x = ((u - 0.5) * 10.0 ** np.round(8 * u - 4)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_bf16_ties_go_to_even():
    one = np.float32(1.0)
    vals = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 1.0 + 2.0 ** -9],
                    dtype=np.float32)
    got = M.bf16_round(vals)
    assert got[0] == 1.0                     # halfway, lower neighbour even
    assert got[1] == 1.0 + 2.0 ** -6         # halfway, upper neighbour even
    assert got[2] == -1.0
    assert got[3] == 1.0                     # below halfway
    assert M.bf16_round(np.array([one]))[0] == 1.0


def test_zero_weights_output_the_last_bias():
    dims, flat, X, T = mlp_case(SEED, 3, 8, 4, 5)
    params = _unpack(dims, flat)
    params = [(np.zeros_like(W), b) for W, b in params]
    Y = M.forward(params, np.array(X).reshape(5, 3))[-1]
    assert np.allclose(Y, params[-1][1][None, :])


def _loss(dims, flat, X, T):
    return M.loss_and_grads(_unpack(dims, flat), X, T)[0]


def test_gradients_match_central_differences():
    dims, flat, X, T = mlp_case(SEED + 1, 3, 5, 4, 6)
    X = np.array(X).reshape(6, 3)
    T = np.array(T).reshape(6, 4)
    flat = np.array(flat)
    loss, grads = M.loss_and_grads(_unpack(dims, flat), X, T)
    g = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    h = 1e-6
    fd = np.empty_like(flat)
    for k in range(flat.size):
        a, b = flat.copy(), flat.copy()
        a[k] += h
        b[k] -= h
        fd[k] = (_loss(dims, a, X, T) - _loss(dims, b, X, T)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.abs(g).max())


def test_gradients_match_torch_autograd():
    dims, flat, X, T = mlp_case(SEED + 2, 5, 16, 7, 9)
    X = np.array(X).reshape(9, 5)
    T = np.array(T).reshape(9, 7)
    params = _unpack(dims, flat)
    loss, grads = M.loss_and_grads(params, X, T)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    h = torch.tensor(X)
    for li, (W, b) in enumerate(tp):
        z = h @ W.T + b
        h = torch.tanh(z) if li < len(tp) - 1 else z
    tl = ((h - torch.tensor(T)) ** 2).sum() / X.shape[0]
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-13 * max(1.0, loss)
    for (dW, db), (W, b) in zip(grads, tp):
        assert np.allclose(dW, W.grad.numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(db, b.grad.numpy(), rtol=1e-12, atol=1e-14)
