"""Nystrom-Gaussian-NFFT eigenvalue approximation (Alg. nystrom_hybrid,
Section 5.2) in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method approximates the k largest eigenpairs of a symmetric operator A
(the paper's A = D^{-1/2} W D^{-1/2}) from 2L products with A:

  step 3  Y = A G for a Gaussian n x L matrix G; Q = orth(Y) by QR;
  step 4  B1 = A Q (n x L), B2 = Q^T B1 (L x L);
  step 5  Sigma_M, U_M: the M largest positive eigenvalues of B2 and their
          orthonormal eigenvectors;
  step 6  QR factorisation Qh Rh = B1 U_M (Qh: n x M, Rh: M x M);
  step 7  eigendecomposition Uh Lambda_M Uh^T = Rh Sigma_M^{-1} Rh^T,
          V_M = Qh Uh;
  step 8  the k largest of Lambda_M and their columns of V_M.

Together these are the eigendecomposition of the rank-M matrix
(A Q) (Q^T A Q)_M^{-1} (A Q)^T, where (.)_M keeps the M largest positive
eigenvalues of Q^T A Q.

Readings where the paper leaves a detail open:
* G is drawn by the caller and passed in (the products depend on it only
  through the range of A G).
* QR factors are taken with a non-negative diagonal of R, which makes them
  unique for full-rank input.
* B2 is symmetrised as (B2 + B2^T)/2 before its eigendecomposition; it is
  symmetric in exact arithmetic.
* "Positive" eigenvalue of B2: larger than POS_REL times the largest
  absolute eigenvalue, so that rounding noise around zero is never inverted.
  If fewer than M qualify, M shrinks to their number; fewer than k is an
  error.
"""
from __future__ import annotations

import numpy as np

POS_REL = 1e-10


def qr_pos(X):
    """Thin QR with a non-negative diagonal of R (Householder via LAPACK)."""
    Q, R = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def positive_top(theta, M: int):
    """Indices of the at most M largest eigenvalues above POS_REL * max|theta|
    (step 5), in descending order of value."""
    theta = np.asarray(theta, dtype=np.float64)
    thr = POS_REL * np.abs(theta).max()
    order = np.argsort(theta)[::-1]
    keep = [int(i) for i in order[:M] if theta[i] > thr]
    return np.array(keep, dtype=np.int64)


def nystrom_gaussian(apply_A, G, k: int, M: int):
    """Alg. nystrom_hybrid, steps 3-8.

    apply_A: maps an (n, c) FP64 block to A times it (steps 1-2, the operator
    set-up and the degrees, live inside it).  G: (n, L) Gaussian matrix.
    Returns (lam (k,) descending, V (n, k) orthonormal, M_used)."""
    G = np.asarray(G, dtype=np.float64)
    n, L = G.shape
    if not (1 <= k <= M <= L <= n):
        raise ValueError("need 1 <= k <= M <= L <= n")
    # step 3
    Y = apply_A(G)
    Q, _ = qr_pos(Y)
    # step 4
    B1 = apply_A(Q)
    B2 = Q.T @ B1
    B2 = 0.5 * (B2 + B2.T)
    # step 5
    theta, U = np.linalg.eigh(B2)
    sel = positive_top(theta, M)
    if len(sel) < k:
        raise ValueError("fewer than k positive eigenvalues in Q^T A Q")
    sig = theta[sel]
    UM = U[:, sel]
    # step 6
    Qh, Rh = qr_pos(B1 @ UM)
    # step 7
    T = Rh @ np.diag(1.0 / sig) @ Rh.T
    lam, Uh = np.linalg.eigh(0.5 * (T + T.T))
    V = Qh @ Uh
    # step 8
    order = np.argsort(lam)[::-1][:k]
    return lam[order], V[:, order], len(sel)


def nystrom_matrix(apply_A, G, M: int):
    """The rank-M Nystrom matrix (A Q)(Q^T A Q)_M^{-1}(A Q)^T formed densely
    (small n only), with Q from an SVD of A G instead of a QR: a second route
    to what steps 6-7 decompose."""
    G = np.asarray(G, dtype=np.float64)
    Y = apply_A(G)
    Uy, s, _ = np.linalg.svd(Y, full_matrices=False)
    Q = Uy[:, s > s[0] * 1e-13]
    C = apply_A(Q)
    theta, U = np.linalg.eigh(0.5 * (Q.T @ C + (Q.T @ C).T))
    sel = positive_top(theta, M)
    F = C @ U[:, sel]
    return F @ np.diag(1.0 / theta[sel]) @ F.T
