"""CPU checks of the per-element gates used by the GPU network tests: an FP32
implementation of the same BF16-operand network (numpy float32 arithmetic,
bf16 rounding of the float32 operands) passes them at the batch sizes the GPU
tests use; planted mistakes in that implementation fail them (one dropped
term in the nodes of one 16-node tile, a wrong sign of one output or of one
gradient element, a node missing from the gradient sums)."""
import numpy as np
import pytest

import mlp_bounds as mb
from oracle import mlp as ref


def bf16_32(a):
    return ref.bf16(a).astype(np.float32)


def fp32_forward(p, X, drop=None):
    P = {k: np.asarray(v, dtype=np.float32) for k, v in ref.unpack(p).items()}
    x = bf16_32(X).T
    z1 = bf16_32(P["W1"]) @ x + P["b1"][:, None]
    if drop is not None:
        z1[3, drop] -= bf16_32(P["W1"])[3, 2] * x[2, drop]
    H1 = np.tanh(z1)
    H2 = np.tanh(bf16_32(P["W2"]) @ bf16_32(H1) + P["b2"][:, None])
    H3 = np.tanh(bf16_32(P["W3"]) @ bf16_32(H2) + P["b3"][:, None])
    return (P["W4"] @ H3 + np.float32(P["b4"])), (H1, H2, H3)


def fp32_grad(p, X, t, skip_last=False):
    P = {k: np.asarray(v, dtype=np.float32) for k, v in ref.unpack(p).items()}
    out, (H1, H2, H3) = fp32_forward(p, X)
    B = X.shape[0]
    g = (np.float32(2.0) * (out - t.astype(np.float32))).astype(np.float32)   # per node
    if skip_last:
        g[-1] = 0.0
    gW4 = H3 @ g
    d3 = P["W4"][:, None] * g[None, :] * (1 - H3 * H3)
    gW3 = bf16_32(d3) @ bf16_32(H2).T
    d2 = (bf16_32(P["W3"]).T @ bf16_32(d3)) * (1 - H2 * H2)
    gW2 = bf16_32(d2) @ bf16_32(H1).T
    d1 = (bf16_32(P["W2"]).T @ bf16_32(d2)) * (1 - H1 * H1)
    gW1 = bf16_32(d1) @ bf16_32(X)
    return (np.concatenate([gW1.ravel(), d1.sum(1), gW2.ravel(), d2.sum(1), gW3.ravel(),
                            d3.sum(1), gW4, [g.sum()]]) * np.float32(1.0 / B)).astype(np.float64)


def net(seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.25, size=ref.NP).astype(np.float32)


def feats(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(B, 16)).astype(np.float32)
    X[:, 8:] = 0.0
    return X


@pytest.mark.parametrize("B", [1, 17, 1000, 4097])
def test_forward_gates_pass_fp32_network_and_catch_mistakes(B):
    p, X = net(3), feats(B, B)
    want, bound, tight = mb.forward_bound(p, X)
    assert np.all(tight <= bound)
    got, _ = fp32_forward(p, X)
    assert mb.forward_gates(got, want, bound, tight) == []
    tile = np.arange(min(B, 16))
    bad, _ = fp32_forward(p, X, drop=tile)
    if B >= 16:
        assert mb.forward_gates(bad, want, bound, tight) != []
    neg = got.copy()
    i = int(np.argmax(np.abs(want) - bound))
    neg[i] = -neg[i]
    assert mb.forward_gates(neg, want, bound, tight) != []


@pytest.mark.parametrize("B", [1, 17, 777, 4097])
def test_gradient_gates_pass_fp32_network_and_catch_mistakes(B):
    p, X = net(5), feats(B, 9 + B)
    t = np.random.default_rng(2).normal(size=B).astype(np.float32)
    L, g_ref, bound, tight, dloss = mb.gradient_bound(p, X, t)
    g = fp32_grad(p, X, t)
    assert mb.gradient_gates(g, g_ref, bound, tight, B) == []
    bad = g.copy()
    big = int(np.argmax(np.abs(g_ref)))
    bad[big] = -bad[big]
    assert mb.gradient_gates(bad, g_ref, bound, tight, B) != []
    if B > 1:
        assert mb.gradient_gates(fp32_grad(p, X, t, skip_last=True), g_ref, bound, tight, B) != []
    S = mb.gradient_abs_sums(p, X, t)
    assert np.all(np.abs(g_ref) <= S * (1 + 1e-9) + 1e-300)
