"""Oracle of the learned expansion-point proposer: FP64 forward and backward of the MLP.

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

Network (the proposer of the greedy, Section 3.3 after Eq. (9), where the next expansion point
is chosen iteratively): x (n_in) -> relu(W1 x + b1) -> relu(W2 . + b2) -> relu(W3 . + b3)
-> logits = W4 . + b4 (n_out); loss = mean over the batch of -log softmax over the allowed
classes (mask > 0) at the label. Parameters are packed as W1 b1 W2 b2 W3 b3 W4 b4 with W_l
row-major (out x in). The weights enter the products rounded to BF16 (nearest even), biases as
given; everything here is computed in FP64.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest BF16 (ties to even), returned as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).copy()
    special = (u & 0x7F800000) == 0x7F800000
    lsb = (u >> 16) & 1
    r = (u + np.uint32(0x7FFF) + lsb) & np.uint32(0xFFFF0000)
    r = np.where(special, u, r).astype(np.uint32)
    return r.view(np.float32)


def layout(n_in, hidden, n_out):
    dims = [(hidden, n_in), (hidden, hidden), (hidden, hidden), (n_out, hidden)]
    out, o = [], 0
    for r, c in dims:
        out.append((o, (r, c)))
        o += r * c
        out.append((o, (r,)))
        o += r
    return out, o


def unpack(params, n_in, hidden, n_out):
    lay, _ = layout(n_in, hidden, n_out)
    return [params[o:o + int(np.prod(sh))].reshape(sh) for o, sh in lay]


def effective(params32, n_in, hidden, n_out):
    """FP64 copy with the weight matrices rounded to BF16 (as the products use them)."""
    p = np.asarray(params32, np.float32).copy()
    lay, _ = layout(n_in, hidden, n_out)
    for k, (o, sh) in enumerate(lay):
        if k % 2 == 0:
            n = int(np.prod(sh))
            p[o:o + n] = bf16_round(p[o:o + n])
    return p.astype(np.float64)


def forward(p, X, n_in, hidden, n_out):
    W = unpack(p, n_in, hidden, n_out)
    a = np.asarray(X, np.float64)
    zs, acts = [], [a]
    for l in range(3):
        z = a @ W[2 * l].T + W[2 * l + 1]
        zs.append(z)
        a = np.maximum(z, 0.0)
        acts.append(a)
    logits = a @ W[6].T + W[7]
    return logits, zs, acts


def loss_and_grad(p, X, labels, mask, n_in, hidden, n_out):
    """Mean masked softmax cross-entropy and its gradient with respect to p (same packing)."""
    W = unpack(p, n_in, hidden, n_out)
    logits, zs, acts = forward(p, X, n_in, hidden, n_out)
    B = logits.shape[0]
    allowed = np.ones_like(logits, bool) if mask is None else np.asarray(mask) > 0
    z = np.where(allowed, logits, -np.inf)
    zmax = z.max(axis=1, keepdims=True)
    e = np.where(allowed, np.exp(z - zmax), 0.0)
    s = e.sum(axis=1, keepdims=True)
    prob = e / s
    lab = np.asarray(labels)
    loss = float(np.mean(-(logits[np.arange(B), lab] - zmax[:, 0] - np.log(s[:, 0]))))
    g = prob.copy()
    g[np.arange(B), lab] -= 1.0
    g /= B
    grads = [None] * 8
    grads[6] = g.T @ acts[3]
    grads[7] = g.sum(axis=0)
    d = g @ W[6]
    for l in (2, 1, 0):
        d = d * (zs[l] > 0)
        grads[2 * l] = d.T @ acts[l]
        grads[2 * l + 1] = d.sum(axis=0)
        d = d @ W[2 * l]
    return loss, np.concatenate([gr.ravel() for gr in grads])
