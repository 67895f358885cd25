"""Power iteration with the factored operator X (+) (X^T (+) w) -- NOT a method of the paper.

Test infrastructure only (see the package docstring).

The paper forms the min-covariance A = (1/N) X (+) X^T first (eq. 5, Alg. 2, Sec. 3.2) and
iterates on A (Alg. 1).  Because (+) is not associative, applying the two factors to w one
after the other, z = X^T (+) w and then X (+) z, is a different operator; it never forms the
D x D matrix and streams X twice per iteration.  It is built as a labelled variant for
comparison, with the same normaliser, residual and stop rule as Alg. 1.

Pins (tests/test_oracle_factored.py):
  * with every |X_ik| >= 1 and ||w||_1 <= 1 each product reduces to a sign matrix product
    (|z_k| <= ||w||_1 <= 1 <= |X_ik|): one step is scale * S (S^T w), S = sign(X), from numpy
    matmul, and the iteration reaches the dominant eigenvector of S S^T (numpy.linalg.eigh);
  * exact rational brute force (fractions.Fraction) on dyadic X with D, N <= 6: z, y and the
    iterates, normalisers and l1 residuals of up to 4 iterations, to float64 rounding;
  * on a generic X the operator differs from Alg. 1 on eq. (5)'s A (non-associativity).
"""
from __future__ import annotations

import numpy as np

from .core import F64, _power_loop, mavp, normalize_l2


def factored_product(X, w, scale=1.0, op="min1"):
    """y = scale * (X (+) (X^T (+) w)) for X of shape D x N (samples as columns, Sec. 1):
    z_k = sum_i op(X_ik, w_i) is the product of column k of X with w, then
    y_i = scale * sum_k op(X_ik, z_k) is the product of row i of X with z."""
    X = np.asarray(X, dtype=F64)
    z = mavp(X.T, w, op)
    return scale * mavp(X, z, op)


def factored_mapi(X, w0, T, tol=0.0, scale=1.0, op="min1", final_l2=False):
    """Iterate w <- y / ||y||_1 with y = factored_product(X, w) (Alg. 1's normalisation,
    residual ||w_t - w_{t-1}||_1 and stop rule), from w0 as given."""
    X = np.asarray(X, dtype=F64)
    res = _power_loop(lambda w: factored_product(X, w, scale, op), w0, T, tol, "l1")
    if final_l2:
        res.w = normalize_l2(res.w)
    return res
