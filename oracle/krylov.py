"""Krylov solvers of Section 4 in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Lanczos (Section 4): q_1 = r/||r||,
  q_{k+1} = (A q_k - alpha_k q_k - beta_k q_{k-1}) / beta_{k+1},
  alpha_k = q_k^T A q_k, beta_{k+1} = ||A q_k - alpha_k q_k - beta_k q_{k-1}||,
  with full reorthogonalisation of every new vector against all previous
  ones (twice, classical Gram-Schmidt).  Ritz pairs come from the
  tridiagonal T_k (eq. krylov1); the residual of a Ritz pair is
  |beta_{k+1} w_k| (the last component of the Ritz vector w of T_k), which is
  the stopping test.  The smallest eigenvalues of L_s are 1 minus the largest
  of A (end of Section 2).
* CG for the kernel-SSL system (I + tau L_s) u = f (eq. ssl::system), stopped
  on the relative recurrence residual ||r_k|| / ||f||.
"""
from __future__ import annotations

import numpy as np


def lanczos_largest(apply, n: int, k: int, tol: float = 1e-10, maxit: int = 300,
                    v0=None, seed: int = 0):
    """k largest eigenpairs of the symmetric operator `apply`.

    Returns (theta descending (k,), Ritz vectors (n, k), residuals (k,), steps)."""
    if v0 is None:
        v0 = np.random.default_rng(seed).standard_normal(n)
    q = np.asarray(v0, dtype=np.float64)
    q = q / np.linalg.norm(q)
    Q = [q]
    alpha, beta = [], []
    for j in range(min(maxit, n)):
        w = apply(Q[j])
        a = float(Q[j] @ w)
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[j - 1] * Q[j - 1]
        Qm = np.stack(Q, axis=1)
        for _ in range(2):
            w = w - Qm @ (Qm.T @ w)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
        theta, S = np.linalg.eigh(T)
        idx = np.argsort(theta)[::-1][:k]
        res = np.abs(b * S[-1, idx])
        if (j + 1 >= k and np.all(res <= tol)) or b == 0.0 or j + 1 == min(maxit, n):
            V = Qm @ S[:, idx]
            return theta[idx], V, res, j + 1
        Q.append(w / b)
    raise AssertionError("unreachable")


def cg(apply_M, f, u0=None, tol: float = 1e-6, maxit: int = 1000):
    """Conjugate gradients for M u = f, M symmetric positive definite.
    Returns (u, iterations, relative recurrence residual)."""
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64)
    r = f - apply_M(u)
    p = r.copy()
    rr = float(r @ r)
    nf = float(np.linalg.norm(f))
    if nf == 0.0:
        return np.zeros_like(f), 0, 0.0
    it = 0
    while np.sqrt(rr) / nf > tol and it < maxit:
        q = apply_M(p)
        a = rr / float(p @ q)
        u = u + a * p
        r = r - a * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return u, it, float(np.sqrt(rr) / nf)
