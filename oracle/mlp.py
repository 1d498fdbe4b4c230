"""FP64 reference of the pointwise warm-start network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network (not from the paper: the learned CG warm start is this build's own
extension): 16 input features -> 64 -> 64 -> 64 -> 1, tanh after the first
three layers, mean squared error loss.  With emulate=True every operand that
the GPU kernels feed to the BF16 matrix cores is rounded to bfloat16
(round-to-nearest-even of its float32 value): the weights W1, W2, W3, the
layer inputs X, H1, H2 in the forward pass, and the deltas (of the summed
squared error, before the mean's 1/B) and layer inputs of the backward
products; all sums, biases, W4 and activations stay FP64.
With emulate=False it is plain FP64 (pinned by finite differences).

Parameter vector (9473): W1[64][16], b1[64], W2[64][64], b2[64], W3[64][64],
b3[64], W4[64], b4.
"""
from __future__ import annotations

import numpy as np

NP = 9473


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) via float32, returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return dict(W1=p[0:1024].reshape(64, 16), b1=p[1024:1088], W2=p[1088:5184].reshape(64, 64),
                b2=p[5184:5248], W3=p[5248:9344].reshape(64, 64), b3=p[9344:9408],
                W4=p[9408:9472], b4=p[9472])


def forward(p, X, emulate=True):
    """Outputs (B,) and activations for features X (B, 16)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.tanh(r(P["W1"]) @ r(X).T + P["b1"][:, None])          # (64, B)
    H2 = np.tanh(r(P["W2"]) @ r(H1) + P["b2"][:, None])
    H3 = np.tanh(r(P["W3"]) @ r(H2) + P["b3"][:, None])
    out = P["W4"] @ H3 + P["b4"]
    return out, (X, H1, H2, H3)


def loss_and_grad(p, X, t, emulate=True):
    """Mean squared error (1/B) sum (out - t)^2 and its gradient (9473,)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(p)
    out, (X, H1, H2, H3) = forward(p, X, emulate)
    B = X.shape[0]
    err = out - np.asarray(t, dtype=np.float64)
    # per-node derivative of the summed squared error; the mean's 1/B is
    # applied to the summed gradient (so the bf16-rounded deltas of a node do
    # not depend on the batch it is in)
    g = 2.0 * err
    gW4 = H3 @ g
    gb4 = g.sum()
    d3 = P["W4"][:, None] * g[None, :] * (1.0 - H3 ** 2)
    gW3 = r(d3) @ r(H2).T
    gb3 = d3.sum(axis=1)
    d2 = (r(P["W3"]).T @ r(d3)) * (1.0 - H2 ** 2)
    gW2 = r(d2) @ r(H1).T
    gb2 = d2.sum(axis=1)
    d1 = (r(P["W2"]).T @ r(d2)) * (1.0 - H1 ** 2)
    gW1 = r(d1) @ r(X)
    gb1 = d1.sum(axis=1)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3, gW4, [gb4]]) / B
    return float(np.mean(err ** 2)), grad
