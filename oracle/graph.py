"""Oracle A: the fully connected Gaussian graph of Section 2 by direct sums.

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64 throughout; the
float32 dataset is promoted exactly, sigma is used in the same coordinates.

Definitions followed (Section 2):
* weights: W_ji = exp(-||v_j - v_i||^2 / sigma^2) for j != i, W_jj = 0
  (eq. W_gaussian); the dense forms also take the other radial kernels of
  eq. W_general (multiquadric, inverse multiquadric);
* degree: d_j = sum_i W_ji, D = diag(d);
* combinatorial Laplacian L = D - W;
* symmetric normalised Laplacian L_s = I - D^{-1/2} W D^{-1/2} (eq. nomlap);
* A = D^{-1/2} W D^{-1/2}, whose largest eigenvalues are 1 minus the
  smallest of L_s (end of Section 2).
"""
from __future__ import annotations

import numpy as np

from . import _ptr, lib


def _v64(v) -> np.ndarray:
    v = np.asarray(v)
    if v.ndim == 1:
        v = v[:, None]
    return np.ascontiguousarray(v.astype(np.float64))


def w_rows(v, sigma: float, x, rows=None) -> np.ndarray:
    """(W x)[rows] by the direct O(n * len(rows)) sum.  x: (n,) or (nvec, n)."""
    V = _v64(v)
    n, d = V.shape
    X = np.asarray(x, dtype=np.float64)
    single = X.ndim == 1
    X = np.ascontiguousarray(X.reshape(1, n) if single else X)
    nvec = X.shape[0]
    R = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(
        np.asarray(rows, dtype=np.int64))
    out = np.empty((nvec, R.shape[0]), dtype=np.float64)
    rc = lib().oracle_w_rows(n, d, _ptr(V), float(sigma), nvec, _ptr(X), R.shape[0], _ptr(R),
                             _ptr(out))
    if rc != 0:
        raise ValueError("oracle_w_rows: bad arguments")
    return out[0] if single else out


def degree(v, sigma: float, rows=None) -> np.ndarray:
    """d_j = sum_{i != j} W_ji for the requested rows (all by default)."""
    V = _v64(v)
    n, d = V.shape
    R = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(
        np.asarray(rows, dtype=np.int64))
    out = np.empty(R.shape[0], dtype=np.float64)
    rc = lib().oracle_degree_rows(n, d, _ptr(V), float(sigma), R.shape[0], _ptr(R), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_degree_rows: bad arguments")
    return out


def apply_W(v, sigma, x):
    return w_rows(v, sigma, x)


def apply_L(v, sigma, x, d=None):
    """L x = D x - W x."""
    d = degree(v, sigma) if d is None else d
    return d * np.asarray(x, dtype=np.float64) - w_rows(v, sigma, x)


def apply_A(v, sigma, x, d=None):
    """A x = D^{-1/2} W D^{-1/2} x."""
    d = degree(v, sigma) if d is None else d
    s = 1.0 / np.sqrt(d)
    return s * w_rows(v, sigma, s * np.asarray(x, dtype=np.float64))


def apply_Ls(v, sigma, x, d=None):
    """L_s x = x - D^{-1/2} W D^{-1/2} x  (eq. nomlap)."""
    x = np.asarray(x, dtype=np.float64)
    return x - apply_A(v, sigma, x, d)


def Ls_rows(v, sigma, x, rows, d):
    """(L_s x)[rows]; needs the full degree vector d (O(n^2) once)."""
    x = np.asarray(x, dtype=np.float64)
    s = 1.0 / np.sqrt(d)
    rows = np.asarray(rows, dtype=np.int64)
    return x[rows] - s[rows] * w_rows(v, sigma, s * x, rows)


# ---- dense forms for small n (a second, independent code path) -------------

def kernel_matrix(v, param: float, kind: str = "gaussian") -> np.ndarray:
    """K(v_i - v_j) for all i, j including the diagonal K(0) (eq. W_general):
    exp(-r^2/param^2) for the Gaussian, sqrt(r^2 + param^2) for the
    multiquadric, 1/sqrt(r^2 + param^2) for the inverse multiquadric kernel,
    exp(-r/param) for the Laplacian RBF kernel (eq. W_laplacian_rbf)
    (small n only)."""
    V = _v64(v)
    diff = V[:, None, :] - V[None, :, :]
    r2 = (diff * diff).sum(axis=2)
    if kind == "gaussian":
        return np.exp(-r2 / (param * param))
    if kind == "multiquadric":
        return np.sqrt(r2 + param * param)
    if kind == "inverse_multiquadric":
        return 1.0 / np.sqrt(r2 + param * param)
    if kind == "laplacian_rbf":
        return np.exp(-np.sqrt(r2) / param)
    raise ValueError(kind)


def dense_W(v, sigma: float, kind: str = "gaussian") -> np.ndarray:
    """The n x n weight matrix formed explicitly (small n only), zero diagonal."""
    W = kernel_matrix(v, sigma, kind)
    np.fill_diagonal(W, 0.0)
    return W


def dense_L(v, sigma, kind: str = "gaussian"):
    W = dense_W(v, sigma, kind)
    return np.diag(W.sum(axis=1)) - W


def dense_Ls(v, sigma, kind: str = "gaussian"):
    W = dense_W(v, sigma, kind)
    s = 1.0 / np.sqrt(W.sum(axis=1))
    return np.eye(W.shape[0]) - s[:, None] * W * s[None, :]


def dense_A(v, sigma, kind: str = "gaussian"):
    W = dense_W(v, sigma, kind)
    s = 1.0 / np.sqrt(W.sum(axis=1))
    return s[:, None] * W * s[None, :]


def smallest_eigs_dense(v, sigma, k):
    """k smallest eigenpairs of L_s by LAPACK (numpy eigh), ascending."""
    lam, U = np.linalg.eigh(dense_Ls(v, sigma))
    return lam[:k], U[:, :k]
