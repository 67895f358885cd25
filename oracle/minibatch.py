"""Mini-batch MAPI with momentum (Algorithm 3, Sec. 3.2).

Test infrastructure only (see the package docstring).

The data X is D x N with the N samples as columns (the layout of eq. 2 and of
the PCA functions here; Algorithm 3 writes the transpose, samples as rows).  The
mini batches are an input: ``batches`` is a T x s integer array of sample
indices, one row per iteration (Algorithm 3 draws them i.i.d.; the draw is the
caller's, so both implementations see the same samples).

Pins (tests/test_oracle_minibatch.py):
  * beta = 0 with every batch holding all N samples reduces Algorithm 3 to
    Algorithm 1 on the min-covariance of eq. (5) with scale 1/N: equal to
    ``mapi(mingram(X, 1/N), w0, T)`` exactly.
  * Sign-aligned data (every sample has the same sign pattern sigma and entries of
    modulus at least one) gives a batch matrix with |A_kl| >= 1 while every iterate
    has ||w||_inf <= ||w||_1 = 1, so A (+) w = sign(A) w = sigma (sigma^T w) exactly
    (the reduction of Sec. 2.1's operator to a matrix product): the momentum
    recurrence and its normalisation are then checked against numpy matmul.
Parity unpinned beyond these: the pseudo-eigenvector of the min-covariance has no
closed form (the paper reports only the 1 - cos^2 curve of Fig. 4).
"""
from __future__ import annotations

import numpy as np

from .core import F64, mavp, normalize_l2, OracleDegenerate
from .pca import mingram


class MinibatchResult:
    def __init__(self):
        self.w = None
        self.iters = 0
        self.norms = []


def minibatch_mapi(X, batches, beta, w0, final_l2=False, op="min1"):
    """Algorithm 3: for t = 0 .. T-1 with batch B_t = batches[t] of s samples,

        A_t     = (1/s) sum_{i in B_t} x_i (+) x_i^T       (eq. 5 on the batch)
        w_{t+1} = A_t (+) w_t - beta w_{t-1}                (w_{-1} = 0)
        nu      = ||w_{t+1}||_1;  w_t <- w_t / nu;  w_{t+1} <- w_{t+1} / nu

    then optionally w_T / ||w_T||_2.  ``op`` "dot" gives the same recurrence with
    ordinary products (the stochastic power method with momentum that Algorithm 3
    modifies).  A zero or non-finite nu raises OracleDegenerate.
    """
    X = np.asarray(X, dtype=F64)
    batches = np.asarray(batches, dtype=np.int64)
    res = MinibatchResult()
    w = np.asarray(w0, dtype=F64).copy()
    w_prev = np.zeros_like(w)
    for B in batches:
        s = len(B)
        A = mingram(np.ascontiguousarray(X[:, B]), 1.0 / s, op)   # same summation as a stored matrix
        y = mavp(A, w, op)
        w_next = y - beta * w_prev
        nu = float(np.sum(np.abs(w_next)))
        if not np.isfinite(nu) or nu == 0.0:
            raise OracleDegenerate(f"normaliser {nu!r} at iteration {res.iters + 1}")
        w_prev = w / nu
        w = w_next / nu
        res.iters += 1
        res.norms.append(nu)
    res.w = normalize_l2(w) if final_l2 else w
    return res
