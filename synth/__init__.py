"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module only draws data: point clouds with the shapes, sizes and value
distributions of the paper's workloads (its own datasets are not available),
random right-hand sides and label vectors.  It contains none of the fast
summation's arithmetic.  Every generator uses numpy's PCG64 ``default_rng`` in
float64 and returns float32 coordinates, which are *the* dataset: both the
HIP library and the oracle receive exactly these values.

All clouds are shifted to their bounding-box midpoint and scaled so that the
largest norm is ``RADIUS`` (= 1/4 - (1/16)/2, the torus ball of the fast
summation with a boundary region of 1/16).  The Gaussian widths quoted for the
workloads are in these output coordinates.
"""
from __future__ import annotations

import numpy as np

RADIUS = 0.21875


def _to_ball(v: np.ndarray) -> np.ndarray:
    """Shift to the bounding-box midpoint, scale to max norm RADIUS, cast f32."""
    v = np.asarray(v, dtype=np.float64)
    c = 0.5 * (v.min(axis=0) + v.max(axis=0))
    v = v - c
    r = np.sqrt((v * v).sum(axis=1)).max()
    if r > 0:
        v = v * (RADIUS / r)
    return np.ascontiguousarray(v.astype(np.float32))


def blobs2d(n: int = 5000, seed: int = 0, centre: float = 0.1, std: float = 0.03):
    """Two isotropic Gaussian blobs in 2-D centred at (+-centre, 0), n/2 each."""
    rng = np.random.default_rng(seed)
    h = n // 2
    a = rng.normal(0.0, std, size=(h, 2)) + np.array([-centre, 0.0])
    b = rng.normal(0.0, std, size=(n - h, 2)) + np.array([centre, 0.0])
    return _to_ball(np.concatenate([a, b], axis=0))


def image_rgb(side: int = 316, regions: int = 6, noise: float = 0.02, seed: int = 0,
              return_labels: bool = False):
    """Piecewise-constant RGB image: Voronoi cells of `regions` uniform sites
    (convex polygons), one U[0,1]^3 colour per region, per-pixel N(0, noise^2).
    Returns the side*side pixel colours as points in d=3."""
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, size=(regions, 2))
    colours = rng.uniform(0.0, 1.0, size=(regions, 3))
    yy, xx = np.meshgrid((np.arange(side) + 0.5) / side, (np.arange(side) + 0.5) / side,
                         indexing="ij")
    pix = np.stack([xx.ravel(), yy.ravel()], axis=1)
    dist = ((pix[:, None, :] - sites[None, :, :]) ** 2).sum(axis=2)
    lab = dist.argmin(axis=1)
    v = colours[lab] + rng.normal(0.0, noise, size=(pix.shape[0], 3))
    out = _to_ball(v)
    return (out, lab) if return_labels else out


def gmm(n: int, d: int = 3, k: int = 10, std_lo: float = 0.005, std_hi: float = 0.03,
        ball: float = 0.15, seed: int = 0, return_labels: bool = False):
    """Gaussian mixture: Dirichlet(1) weights, centres uniform in a ball of
    radius `ball`, isotropic std U[std_lo, std_hi] per component."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(k))
    dirs = rng.normal(size=(k, d))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rad = ball * rng.uniform(0.0, 1.0, size=k) ** (1.0 / d)
    centres = dirs * rad[:, None]
    stds = rng.uniform(std_lo, std_hi, size=k)
    counts = rng.multinomial(n, w)
    lab = np.repeat(np.arange(k), counts)
    v = centres[lab] + rng.normal(size=(n, d)) * stds[lab][:, None]
    out = _to_ball(v)
    return (out, lab) if return_labels else out


def moons_and_roll(n: int = 1_000_000, seed: int = 1, noise: float = 0.01):
    """Three classes of n/3 points in 3-D: two interleaved crescents (half
    circles of radius 0.12 in the plane z=0, offset like the two-moons set)
    and a Swiss roll (spiral sheet) beside them, isotropic noise `noise`.
    Returns (points f32 (n,3), labels int64 (n,))."""
    rng = np.random.default_rng(seed)
    c = n // 3
    sizes = [c, c, n - 2 * c]
    r = 0.12
    t0 = rng.uniform(0.0, np.pi, size=sizes[0])
    a = np.stack([r * np.cos(t0) - 0.12, r * np.sin(t0) - 0.03, np.zeros_like(t0)], axis=1)
    t1 = rng.uniform(0.0, np.pi, size=sizes[1])
    b = np.stack([r - r * np.cos(t1) - 0.12, 0.5 * r - r * np.sin(t1) - 0.03,
                  np.zeros_like(t1)], axis=1)
    t2 = rng.uniform(1.5 * np.pi, 4.5 * np.pi, size=sizes[2])
    h = rng.uniform(-0.08, 0.08, size=sizes[2])
    s = 0.0065
    roll = np.stack([s * t2 * np.cos(t2) + 0.15, h, s * t2 * np.sin(t2)], axis=1)
    v = np.concatenate([a, b, roll], axis=0) + rng.normal(0.0, noise, size=(n, 3))
    lab = np.repeat(np.arange(3), sizes)
    return _to_ball(v), lab


def spirals(n: int, classes: int = 5, seed: int = 0, height: float = 10.0,
            radius: float = 2.0, turns: float = 1.5, noise: float = 0.15):
    """Interleaved 3-D spiral arms, one class per arm, n / classes points each
    (the first n % classes arms get one more).  Arm c at parameter t ~ U[0, 1]:
    angle 2 pi (turns t + c / classes), distance from the axis
    radius (0.25 + t), height `height` t, plus N(0, noise^2) per coordinate.
    Returns (points f32 in the ball, labels, scale) with `scale` the factor
    from the generator's units to the returned coordinates (a width quoted in
    generator units times `scale` is the width for the returned points)."""
    rng = np.random.default_rng(seed)
    sizes = [n // classes + (1 if c < n % classes else 0) for c in range(classes)]
    parts = []
    for c, m in enumerate(sizes):
        t = rng.uniform(0.0, 1.0, size=m)
        ang = 2.0 * np.pi * (turns * t + c / classes)
        rad = radius * (0.25 + t)
        parts.append(np.stack([rad * np.cos(ang), rad * np.sin(ang), height * t], axis=1))
    v = np.concatenate(parts, axis=0) + rng.normal(0.0, noise, size=(n, 3))
    c0 = 0.5 * (v.min(axis=0) + v.max(axis=0))
    r = np.sqrt(((v - c0) ** 2).sum(axis=1)).max()
    lab = np.repeat(np.arange(classes), sizes)
    return _to_ball(v), lab, RADIUS / r


def batched_clouds(count: int = 64, seed: int = 0, n_lo: int = 1000, n_hi: int = 200_000,
                   d: int = 3):
    """`count` independent Gaussian-mixture clouds: n log-uniform in
    [n_lo, n_hi], 3..8 components, std U[0.01, 0.05], sigma U[0.03, 0.15].
    Returns a list of (points f32, sigma)."""
    out = []
    for g in range(count):
        rng = np.random.default_rng([seed, g])
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        k = int(rng.integers(3, 9))
        sigma = float(rng.uniform(0.03, 0.15))
        sub = int(rng.integers(0, 2**31 - 1))
        out.append((gmm(n, d=d, k=k, std_lo=0.01, std_hi=0.05, seed=sub), sigma))
    return out


def uniform_ball(n: int, d: int = 3, seed: int = 0):
    """Uniform points in the ball (least clustered reference cloud)."""
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n, d))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rad = rng.uniform(0.0, 1.0, size=n) ** (1.0 / d)
    return _to_ball(dirs * rad[:, None])


def normal_vectors(n: int, nvec: int = 1, seed: int = 12345, dtype=np.float32):
    """x ~ N(0, 1), shape (n,) for nvec == 1 else (nvec, n) (one vector per row)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(size=(nvec, n))
    x = x.astype(dtype)
    return x[0] if nvec == 1 else np.ascontiguousarray(x)


def ssl_rhs(labels: np.ndarray, cls: int, frac: float = 0.02, seed: int = 0):
    """One-vs-rest training vector f in {-1, 0, +1}: a uniformly drawn `frac`
    of the nodes is labelled, +1 where the label is `cls`, -1 otherwise."""
    rng = np.random.default_rng(seed)
    n = labels.shape[0]
    k = max(1, int(round(frac * n)))
    idx = rng.choice(n, size=k, replace=False)
    f = np.zeros(n, dtype=np.float64)
    f[idx] = np.where(labels[idx] == cls, 1.0, -1.0)
    return f
