"""PCA forms: covariance (eq. 2), min-covariance (eq. 5), deflation, top-k extraction.

Test infrastructure only (see the package docstring).

Pins (tests/test_oracle_pca.py):
  * mingram: diagonal entries equal scale * ||x_i||_1 exactly (the l1 identity of
    Sec. 2.1); symmetry; for X with entries of modulus one the min-covariance
    equals scale * X X^T from numpy matmul.
  * deflate_projection / pca_topk with method "rpi": the top-k eigenvectors of
    numpy.linalg.eigh on planted-gap covariance matrices, and P^T P = I.
Parity unpinned: pca_topk with method "mapi" beyond those invariants (the
pseudo-eigenvectors of the min-covariance have no closed form).
"""
from __future__ import annotations

import numpy as np

from .core import F64, TERMS, mapi, rpi

def covariance(X, scale):
    """Sample covariance of eq. (2): scale * X X^T, X of shape D x N (samples as columns)."""
    X = np.asarray(X, dtype=F64)
    return scale * (X @ X.T)


def mingram(X, scale, op="min1"):
    """Min-covariance of eq. (5): A_ij = scale * (x_i^T (+) x_j), x_i the i-th row of X.

    X is D x N with the N samples as columns (Sec. 1, eq. 2), so row i of X holds
    coordinate i of every sample and A is D x D.  Every entry is formed, not only
    one triangle, so that symmetry can be tested.
    """
    X = np.asarray(X, dtype=F64)
    term = TERMS[op]
    D = X.shape[0]
    A = np.empty((D, D), dtype=F64)
    for i in range(D):
        A[i, :] = scale * np.sum(term(X[i][None, :], X), axis=1)
    return A


def mingram_entry(X, i, j, scale, op="min1"):
    """One entry of eq. (5), for sampled checks of large builds."""
    X = np.asarray(X, dtype=F64)
    return float(scale * np.sum(TERMS[op](X[i], X[j])))


def deflate_projection(A, P):
    """(I - sum_k p_k p_k^T) A, the deflated matrix of Sec. 1 (P has orthonormal columns)."""
    A = np.asarray(A, dtype=F64)
    if P is None or P.shape[1] == 0:
        return A.copy()
    P = np.asarray(P, dtype=F64)
    return A - P @ (P.T @ A)


def _mgs_append(P, w):
    """l2-normalise w (Sec. 2.2: the final MAPI vector is l2-normalised before later
    vectors are extracted) and orthogonalise it against the columns of P by modified
    Gram-Schmidt, so that sum_k p_k p_k^T stays a projector.  The paper is silent on
    the orthogonalisation; MAPI vectors are not orthogonal by themselves."""
    p = np.asarray(w, dtype=F64)
    p = p / np.sqrt(np.sum(p * p))
    for l in range(P.shape[1]):
        p = p - np.sum(P[:, l] * p) * P[:, l]
    p = p / np.sqrt(np.sum(p * p))
    return np.concatenate([P, p[:, None]], axis=1)


def pca_topk(X, k, W0, method="mapi", T=100, tol=0.0, scale=None, op="min1", A=None):
    """Top-k principal (pseudo-)vectors with deflation.

    method "mapi": power iteration of eq. (6) on the min-covariance of eq. (5).
    method "rpi":  power iteration of eq. (1) on the covariance of eq. (2).
    Vector i is extracted from (I - P P^T) A where P holds the i-1 earlier vectors
    (Sec. 1), started from column i of W0 (D x k).  Returns (P, [IterResult]).
    ``A`` may pass a prebuilt matrix of the right kind to skip the build.  ``T`` is
    one iteration limit for every vector or a sequence of k limits, one per vector.
    """
    X = np.asarray(X, dtype=F64)
    D, N = X.shape
    if scale is None:
        scale = 1.0 / N
    if A is None:
        A = mingram(X, scale, op) if method == "mapi" else covariance(X, scale)
    W0 = np.asarray(W0, dtype=F64)
    P = np.zeros((D, 0), dtype=F64)
    Ts = [int(T)] * k if np.isscalar(T) else [int(t) for t in T]
    results = []
    for i in range(k):
        Ai = deflate_projection(A, P)
        if method == "mapi":
            r = mapi(Ai, W0[:, i], Ts[i], tol, op=op)
        else:
            r = rpi(Ai, W0[:, i], Ts[i], tol, norm="l2")
        results.append(r)
        P = _mgs_append(P, r.w)
    return P, results
