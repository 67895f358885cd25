"""Image reconstruction via MAPI (Algorithm 2, Sec. 3.1).

Test infrastructure only (see the package docstring).

Pins (tests/test_oracle_image.py):
  * min_outer: the diagonal of W (+) W^T is sum_k |W_jk| (the l1 identity of Sec. 2.1),
    the matrix is symmetric, and for columns of constant modulus c it equals
    c * sign(W) sign(W)^T (numpy matmul).
  * minouter_deflate and minouter_reconstruct (Alg. 2, deflation and reconstruction steps):
    for vectors of constant modulus, where w (+) w^T = c s s^T, they equal the numpy
    expressions C - c s (s^T C) and sum_k c_k s_k (s_k^T Vc) + m -- which fixes the side
    the min-outer product multiplies from (a transposed product fails).
  * image_reconstruct with method "mapi": its vectors are oracle.mapi on the eq. (5)
    min-covariance with the 1/(N-1) scale and on the deflated matrix, and R is the
    reconstruction step applied to them (checked by composing the pinned steps).
  * image_reconstruct with method "rpi": the two vectors span the top-2 eigenspace of the
    covariance (numpy.linalg.eigh) and the reconstruction equals the projection of every
    centred image onto that space plus the mean.
Parity unpinned: none beyond the MAPI fixed point (see core).
"""
from __future__ import annotations

import numpy as np

from .core import F64, term_min1, TERMS, mapi, rpi, normalize_l2
from .pca import covariance, mingram


def min_outer(W, op="min1"):
    """(W (+) W^T)_jl = sum_k op(W_jk, W_lk): the matrix extension (Sec. 2.1) of W W^T for W of
    shape P x K (a vector is one column)."""
    W = np.asarray(W, dtype=F64)
    if W.ndim == 1:
        W = W[:, None]
    term = TERMS[op]
    M = np.zeros((W.shape[0], W.shape[0]), dtype=F64)
    for k in range(W.shape[1]):
        M += term(W[:, k][:, None], W[:, k][None, :])
    return M


def minouter_deflate(C, w, op="min1"):
    """Alg. 2, deflation step: C - (w (+) w^T) C, the min-outer product of the first vector
    multiplying C from the left."""
    C = np.asarray(C, dtype=F64)
    return C - min_outer(w, op) @ C


def minouter_reconstruct(W, Vc, m, op="min1"):
    """Alg. 2, reconstruction step: (W (+) W^T) Vc + m, the min-outer product of the vectors
    (columns of W) applied to the centred images (columns of Vc), plus the mean image m."""
    Vc = np.asarray(Vc, dtype=F64)
    return min_outer(W, op) @ Vc + np.asarray(m, dtype=F64)[:, None]


def image_reconstruct(V, T, w0, method="mapi", op="min1", tol=0.0):
    """Algorithm 2 on the P x N matrix V whose columns are the N corrupted images:

      m = mean of the columns; Vc = V - m
      C = (1/(N-1)) Vc (+) Vc^T             (line 4; the covariance of eq. 2 for RPI)
      w1 = dominant vector of C             (line 5)
      w2 = dominant vector of C - (w1 (+) w1^T) C      (line 6; RPI: the projection C - w1 w1^T C)
      W = [w1 w2];  R = (W (+) W^T) Vc + m  (line 8; RPI: W W^T Vc + m)

    Each vector is the result of T iterations (tolerance tol) from w0 of MAPI (eq. 6, product
    `op`) as Algorithm 1 returns it -- l1-normalised, without the optional l2 step -- or of RPI
    (eq. 1), l2-normalised.  The l1 norm is the unit of the operator's geometry (w (+) w =
    ||w||_1, Sec. 2.1): with ||w||_1 = 1 and entries of similar modulus, (w (+) w^T) w ~ w, as
    w w^T w = w for a unit l2 vector; with l2-normalised MAPI vectors the extension of W W^T is
    larger by about sqrt(P).  Returns (R, W, (result 1, result 2)).
    """
    V = np.asarray(V, dtype=F64)
    N = V.shape[1]
    m = V.mean(axis=1)
    Vc = V - m[:, None]
    mapi_like = method == "mapi"
    C = mingram(Vc, 1.0 / (N - 1), op) if mapi_like else covariance(Vc, 1.0 / (N - 1))

    def solve(A):
        if mapi_like:
            return mapi(A, w0, T, tol, op=op)
        return rpi(A, w0, T, tol, final_l2=True)

    r1 = solve(C)
    w1 = r1.w
    C2 = minouter_deflate(C, w1, op) if mapi_like else C - np.outer(w1, w1) @ C
    r2 = solve(C2)
    W = np.stack([w1, r2.w], axis=1)
    R = minouter_reconstruct(W, Vc, m, op) if mapi_like else W @ W.T @ Vc + m[:, None]
    return R, W, (r1, r2)


def psnr(x, ref, peak=1.0):
    """Peak signal-to-noise ratio in dB of x against ref (Table 1)."""
    x = np.asarray(x, dtype=F64)
    ref = np.asarray(ref, dtype=F64)
    mse = float(np.mean((x - ref) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(peak * peak / mse)
