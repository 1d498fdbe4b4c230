"""Kernel ridge regression (Section 6.3) in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The dual coefficients solve (K + beta I) alpha = f with the Gram matrix
K_ij = K(x_i - x_j), diagonal K(0) included, for a radial kernel of eq.
W_general; the prediction at a point x is F(x) = sum_i alpha_i K(x_i - x).
Here K is formed densely and the system is solved by LAPACK (the definition);
small n only.
"""
from __future__ import annotations

import numpy as np

from . import graph


def gram(v, param: float, kind: str = "gaussian") -> np.ndarray:
    """K_ij = K(v_i - v_j), diagonal included."""
    return graph.kernel_matrix(v, param, kind)


def solve(v, param: float, beta: float, f, kind: str = "gaussian") -> np.ndarray:
    """alpha = (K + beta I)^{-1} f."""
    K = gram(v, param, kind)
    return np.linalg.solve(K + beta * np.eye(K.shape[0]), np.asarray(f, dtype=np.float64))


def predict(v, alpha, x_new, param: float, kind: str = "gaussian") -> np.ndarray:
    """F(x) = sum_i alpha_i K(v_i - x) at the rows of x_new."""
    V = np.asarray(v, dtype=np.float64)
    X = np.asarray(x_new, dtype=np.float64)
    d2 = ((X[:, None, :] - V[None, :, :]) ** 2).sum(axis=2)
    if kind == "gaussian":
        Kx = np.exp(-d2 / (param * param))
    elif kind == "multiquadric":
        Kx = np.sqrt(d2 + param * param)
    elif kind == "laplacian_rbf":
        Kx = np.exp(-np.sqrt(d2) / param)
    else:
        Kx = 1.0 / np.sqrt(d2 + param * param)
    return Kx @ np.asarray(alpha, dtype=np.float64)
