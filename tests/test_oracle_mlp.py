"""Pins of the MLP oracle: central finite differences of the FP64 loss, BF16 rounding, and the
softmax cross-entropy identity d loss / d logits = (p - onehot) / batch."""
import numpy as np

import workloads as W
from oracle import mlp


def _net(n_in=7, hidden=5, n_out=6, seed=11):
    _, n = mlp.layout(n_in, hidden, n_out)
    rng = W.SplitMix64(seed)
    p = (rng.uniforms(n) - 0.5)
    return p, n_in, hidden, n_out


def test_finite_differences():
    p, n_in, H, n_out = _net()
    rng = W.SplitMix64(5)
    B = 4
    X = rng.uniforms(B * n_in).reshape(B, n_in) - 0.5
    labels = np.array([0, 3, 5, 2])
    mask = np.ones((B, n_out))
    mask[1, 1] = 0
    mask[2, 4] = 0
    loss, g = mlp.loss_and_grad(p, X, labels, mask, n_in, H, n_out)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(len(p)):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd[k] = (mlp.loss_and_grad(pp, X, labels, mask, n_in, H, n_out)[0]
                 - mlp.loss_and_grad(pm, X, labels, mask, n_in, H, n_out)[0]) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_logit_gradient_identity():
    # a network whose last layer is the identity on a one-hot hidden state exposes dL/dlogits
    n_in, H, n_out = 3, 3, 3
    lay, n = mlp.layout(n_in, H, n_out)
    p = np.zeros(n)
    Wm = mlp.unpack(p, n_in, H, n_out)
    for l in range(4):
        np.fill_diagonal(Wm[2 * l], 1.0)
    p = np.concatenate([w.ravel() for w in Wm])
    X = np.array([[0.2, 1.0, 0.5]])
    loss, g = mlp.loss_and_grad(p, X, np.array([2]), None, n_in, H, n_out)
    z = X[0]
    prob = np.exp(z) / np.exp(z).sum()
    assert np.isclose(loss, -np.log(prob[2]))
    gb4 = g[lay[7][0]:lay[7][0] + n_out]
    assert np.allclose(gb4, prob - np.eye(3)[2])


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e38, np.inf], np.float32)
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0                # tie to even (mantissa LSB 0)
    assert r[2] == np.float32(1.0 + 2 ** -7)          # above the tie: rounds up
    assert r[3] == -2.5 and np.isinf(r[5])
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
