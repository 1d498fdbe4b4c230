"""Per-element error bounds for the BF16 matrix-core network against the
BF16-emulated FP64 reference (oracle.mlp with emulate=True).

The GPU and the reference round the same operands to bfloat16; they differ by
(a) FP32 accumulation of the dot products (the products of two bf16 values
are exact in FP32), (b) the FP32 tanh, and (c) bf16 rounding of operands the
GPU computed (activations, deltas): where the GPU's FP32 value and the
reference's value lie on different sides of a bf16 rounding boundary, the two
rounded operands differ by about one bf16 ulp.

Two tiers, both rigorous:
* A node is a "flip candidate" if one of its bf16-rounded operands (any
  layer; for gradients also the deltas) lies within its FP32 error bound of a
  rounding boundary, the bounds propagated without flips.  At every other
  node no operand can flip: by induction over the layers its errors stay at
  the no-flip bounds, so its outputs get the tight FP32-level bound.
* At candidate nodes every operand within its (larger, propagated) bound of
  a boundary may flip, and those bounds cascade through the later layers.

Gradients sum over nodes; each node contributes with its own tier.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp as ref

U32 = 2.0 ** -24          # FP32 unit roundoff
TANH_ABS = 2.0 ** -20     # FP32 tanh, absolute error allowance for |tanh| <= 1


def _gamma(k: int) -> float:
    """Bound on the relative error of a k-term FP32 sum (Higham's gamma_k,
    with a few extra terms for the bias and the final rounding)."""
    return (k + 4) * U32 / (1.0 - (k + 4) * U32)


def bf16_flip_room(x: np.ndarray) -> tuple:
    """(a lower bound on the distance of x to the nearest bf16 rounding
    boundary, one bf16 ulp at x).  With lo <= |x| < hi the neighbouring bf16
    values, the boundaries nearby are the midpoint (lo + hi)/2 and, below lo,
    one at least a quarter ulp away (half the ulp of the binade below)."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    bits = ax.astype(np.float32).view(np.uint32)
    lo = (bits & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    hi = ((bits & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    ulp = hi - lo
    room = np.minimum(np.abs(ax - 0.5 * (lo + hi)), np.abs(ax - lo) + 0.25 * ulp)
    return room, ulp


def _propagate(p, X, t, flips: bool):
    """Per-node bounds of every intermediate (columns = nodes).  flips=False:
    no operand flips (valid at non-candidate nodes); flips=True: any operand
    within its bound of a boundary may flip.  Also returns, per node, whether
    some operand lies within its bound of a boundary."""
    P = ref.unpack(p)
    r = ref.bf16
    out, (Xa, H1, H2, H3) = ref.forward(p, X, emulate=True)
    B = X.shape[0]
    near_any = np.zeros(B, dtype=bool)

    def rop(x, dx):
        nonlocal near_any
        room, ulp = bf16_flip_room(x)
        near = dx >= room
        near_any |= near.any(axis=0)
        # a flip: dx plus the two half-ulp rounding errors (one ulp, two at a binade edge)
        return np.where(near, dx + 2.0 * ulp, 0.0) if flips else np.zeros_like(dx)

    def layer(Wr, hr, dhr, b, k):
        S = np.abs(Wr) @ np.abs(hr) + np.abs(b)[:, None]
        return np.abs(Wr) @ dhr + _gamma(k) * S

    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    x = r(Xa).T                                   # (16, B): both round the same float32 input
    o = {"out": out, "H": (H1, H2, H3), "x": x}
    dh1 = layer(W1, x, np.zeros_like(x), P["b1"], 16) + TANH_ABS
    dr1 = rop(H1, dh1)
    dh2 = layer(W2, r(H1), dr1, P["b2"], 64) + TANH_ABS
    dr2 = rop(H2, dh2)
    dh3 = layer(W3, r(H2), dr2, P["b3"], 64) + TANH_ABS
    S4 = np.abs(P["W4"]) @ np.abs(H3) + abs(P["b4"])
    o["dout"] = np.abs(P["W4"]) @ dh3 + _gamma(64) * S4
    o.update(dh1=dh1, dh2=dh2, dh3=dh3, dr1=dr1, dr2=dr2)
    if t is not None:
        err = out - np.asarray(t, dtype=np.float64)
        g = 2.0 * err                 # per node, before the mean's 1/B (as the kernels round)
        dg = 2.0 * o["dout"] + _gamma(4) * np.abs(g)
        W4 = P["W4"][:, None]
        f3 = 1.0 - H3 ** 2
        d3 = W4 * g[None, :] * f3
        dd3 = np.abs(W4) * (dg[None, :] * f3 + np.abs(g)[None, :] * 2.0 * np.abs(H3) * dh3
                            + 4 * U32 * np.abs(g)[None, :])
        rd3 = rop(d3, dd3)
        s2 = W3.T @ r(d3)
        ds2 = np.abs(W3).T @ rd3 + _gamma(64) * (np.abs(W3).T @ np.abs(r(d3)))
        f2 = 1.0 - H2 ** 2
        d2 = s2 * f2
        dd2 = ds2 * f2 + np.abs(s2) * 2.0 * np.abs(H2) * dh2 + 4 * U32 * np.abs(d2)
        rd2 = rop(d2, dd2)
        s1 = W2.T @ r(d2)
        ds1 = np.abs(W2).T @ rd2 + _gamma(64) * (np.abs(W2).T @ np.abs(r(d2)))
        f1 = 1.0 - H1 ** 2
        d1 = s1 * f1
        dd1 = ds1 * f1 + np.abs(s1) * 2.0 * np.abs(H1) * dh1 + 4 * U32 * np.abs(d1)
        rd1 = rop(d1, dd1)
        o.update(err=err, g=g, dg=dg, d=(d1, d2, d3), dd=(dd1, dd2, dd3), rd=(rd1, rd2, rd3))
    o["near"] = near_any
    return o


def forward_bound(p, X):
    """(reference outputs (B,), per-node bound on |GPU - reference| (B,),
    per-node bound if no operand flips (B,))."""
    a = _propagate(p, X, None, flips=False)
    b = _propagate(p, X, None, flips=True)
    cand = a["near"]
    return a["out"], np.where(cand, b["dout"], a["dout"]), a["dout"]


def gradient_abs_sums(p, X, t):
    """Per gradient element, the sum over nodes of the absolute values of the
    nodes' contributions (the scale of FP32 summation errors over nodes)."""
    r = ref.bf16
    a = _propagate(p, X, t, flips=False)
    H1, H2, H3 = a["H"]
    g = np.abs(a["g"])
    d1, d2, d3 = (np.abs(v) for v in a["d"])
    x = np.abs(a["x"])
    return np.concatenate([(np.abs(r(d1)) @ x.T).ravel(), d1.sum(1),
                           (np.abs(r(d2)) @ np.abs(r(H1)).T).ravel(), d2.sum(1),
                           (np.abs(r(d3)) @ np.abs(r(H2)).T).ravel(), d3.sum(1),
                           np.abs(H3) @ g, [g.sum()]]) / X.shape[0]


def gradient_bound(p, X, t):
    """(reference loss, reference gradient (9473,), per-element bound on the
    gradient difference (9473,), the same bound if no operand flips anywhere
    (9473,), bound on the loss difference)."""
    B = X.shape[0]
    L, g_ref = ref.loss_and_grad(p, X, t, emulate=True)
    a = _propagate(p, X, t, flips=False)
    b = _propagate(p, X, t, flips=True)
    bound, dloss = _grad_sums(a, b, a["near"], B)
    tight, _ = _grad_sums(a, a, np.zeros(B, dtype=bool), B)
    # the sums are of per-node contributions; the GPU then multiplies by
    # fl(1/B) in FP32 (two roundings)
    def scaled(x):
        return x / B + 3.0 * U32 * (np.abs(g_ref) + x / B)
    return L, g_ref, scaled(bound), scaled(tight), dloss


def _grad_sums(a, b, cand, B):
    r = ref.bf16

    def pick(key, i=None):
        va, vb = (a[key], b[key]) if i is None else (a[key][i], b[key][i])
        return np.where(cand, vb, va) if va.ndim == 1 else np.where(cand[None, :], vb, va)

    H1, H2, H3 = a["H"]
    g, err = a["g"], a["err"]
    dout, dg = pick("dout"), pick("dg")
    dh3 = pick("dh3")
    dr1, dr2 = pick("dr1"), pick("dr2")
    d1, d2, d3 = a["d"]
    dd1, dd2, dd3 = pick("dd", 0), pick("dd", 1), pick("dd", 2)
    rd1, rd2, rd3 = pick("rd", 0), pick("rd", 1), pick("rd", 2)
    dloss = (2.0 * np.abs(err) * dout + dout ** 2).sum() / B + _gamma(B) * float(np.mean(err ** 2))
    gB = _gamma(B + 64)
    h2r, h1r, xr = r(H2), r(H1), a["x"]
    # last layer: gW4 = H3 g, gb4 = sum g (FP32 sums over the B nodes)
    dW4 = dh3 @ np.abs(g) + np.abs(H3) @ dg + gB * (np.abs(H3) @ np.abs(g))
    db4 = dg.sum() + gB * np.abs(g).sum()
    # gW3 = r(d3) r(H2)^T, gb3 = sum d3, and so on down the layers
    dW3 = rd3 @ np.abs(h2r).T + np.abs(r(d3)) @ dr2.T + gB * (np.abs(r(d3)) @ np.abs(h2r).T)
    db3 = dd3.sum(axis=1) + gB * np.abs(d3).sum(axis=1)
    dW2 = rd2 @ np.abs(h1r).T + np.abs(r(d2)) @ dr1.T + gB * (np.abs(r(d2)) @ np.abs(h1r).T)
    db2 = dd2.sum(axis=1) + gB * np.abs(d2).sum(axis=1)
    dW1 = rd1 @ np.abs(xr).T + gB * (np.abs(r(d1)) @ np.abs(xr).T)
    db1 = dd1.sum(axis=1) + gB * np.abs(d1).sum(axis=1)
    bound = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3, dW4, [db4]])
    return bound, dloss


def forward_gates(got, want, bound, tight):
    """The forward checks: every output within its rigorous bound, and at most
    2 + B/100 outputs beyond the no-flip bound (an FP32 implementation flips a
    bf16 operand at ~0.05% of the nodes).  Returns a list of failures."""
    e = np.abs(np.asarray(got, dtype=np.float64) - want)
    fails = []
    if not np.all(e <= bound):
        i = int(np.argmax(e - bound))
        fails.append("node %d: |err| %.3g > bound %.3g" % (i, e[i], bound[i]))
    k = int((e > tight).sum())
    if k > 2 + len(e) // 100:
        fails.append("%d of %d outputs beyond the no-flip bound" % (k, len(e)))
    return fails


def gradient_gates(got, want, bound, tight, batch=None):
    """The gradient checks: every element within its rigorous bound, and at
    most 5% of the elements beyond the no-flip bound.  Below 64 nodes one
    bf16 flip of one node's delta already moves a whole row of a weight
    gradient (and, through the next layer's deltas, more) beyond the no-flip
    bound, so there the second gate allows half of the elements and the
    rigorous bound decides."""
    e = np.abs(np.asarray(got, dtype=np.float64) - want)
    fails = []
    if not np.all(e <= bound):
        i = int(np.argmax(e - bound))
        fails.append("element %d: |err| %.3g > bound %.3g" % (i, e[i], bound[i]))
    frac = float((e > tight).mean())
    if frac > (0.05 if batch is None or batch >= 64 else 0.5):
        fails.append("%.1f%% of the elements beyond the no-flip bound" % (100 * frac))
    return fails
