"""Operators, the MAVP matrix-vector product, MAPI (Algorithm 1) and RPI (eq. 1).

Test infrastructure only (see the package docstring).

Pins (tests/test_oracle_core.py):
  * term_min1 / vec_product: the l1 identity x (+) x = ||x||_1 (Sec. 2.1, text
    after eq. 4), symmetry, odd sign symmetry, joint positive homogeneity,
    min1 = min2(a,b) - min2(-a,b), permutation invariance.
  * mavp: the sign(A) reduction -- when every |A_ij| >= 1 >= |w_j| the product
    equals the ordinary product sign(A) @ w (numpy matmul), on non-symmetric A,
    which fixes the row/column orientation.
  * mapi: the iterates keep ||w_t||_1 = 1 (Sec. 2.2); on a sign-dominated matrix
    MAPI is l1-normalised power iteration on sign(A) and converges to the
    dominant eigenvector from numpy.linalg.eigh; a constant matrix reaches 1/n
    in one step; Proposition 1's closed form with the diamond operator of
    eq. (7), reached exactly at the second iteration.
  * rpi: the dominant eigenvector of numpy.linalg.eigh on planted-gap matrices.
  * mavp, mapi, rpi (l1 form): exact rational brute force (fractions.Fraction) on
    dyadic systems with n <= 8 for up to 5 iterations -- the product exactly, and the
    iterates, the l1 normalisers and the l1 residual sequence ||w_t - w_{t-1}||_1 to
    float64 rounding (tests/test_oracle_bruteforce.py), including the stop iteration
    for a tolerance between two exact residuals.
  * ranks: the rank lists the paper prints for its own vectors (Sec. 3.2 and
    Sec. 3.3), stored under tests/golden/.
Parity unpinned: MAPI's fixed point on general matrices (no closed form exists;
the paper leaves convergence for general operators open, Sec. 2.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

F64 = np.float64


class OracleDegenerate(ArithmeticError):
    """The normaliser of an iterate is zero or not finite (the paper is silent)."""


# --------------------------------------------------------------------------
# Element terms of the vector products
# --------------------------------------------------------------------------
def term_min1(a, b):
    """One term of the min1 product, eq. (3): sign(a b) * min(|a|, |b|).

    sign(a b) is written as sign(a) * sign(b), equal for real numbers, so that a
    product underflowing to zero cannot zero the sign.
    """
    a = np.asarray(a, dtype=F64)
    b = np.asarray(b, dtype=F64)
    return np.sign(a) * np.sign(b) * np.minimum(np.abs(a), np.abs(b))


def term_min2(a, b):
    """One term of the min2 product, eq. (4): 1(sign a = sign b) * min(|a|, |b|)."""
    a = np.asarray(a, dtype=F64)
    b = np.asarray(b, dtype=F64)
    return np.where(np.sign(a) == np.sign(b), np.minimum(np.abs(a), np.abs(b)), 0.0)


def term_diamond(a, b):
    """One term of the additive operator of eq. (7): sign(a) b + a sign(b).

    The printed equation names its operands x, y while the left side names w, x;
    this reads them as the two vectors being multiplied.
    """
    a = np.asarray(a, dtype=F64)
    b = np.asarray(b, dtype=F64)
    return np.sign(a) * b + a * np.sign(b)


def term_dot(a, b):
    """One term of the Euclidean inner product used by regular power iteration, eq. (1)."""
    return np.asarray(a, dtype=F64) * np.asarray(b, dtype=F64)


TERMS = {"min1": term_min1, "min2": term_min2, "diamond": term_diamond, "dot": term_dot}


def vec_product(w, x, op="min1"):
    """w^T (+) x = sum_i term(w_i, x_i), eqs. (3), (4), (7)."""
    return float(np.sum(TERMS[op](w, x)))


def mavp(A, w, op="min1"):
    """Matrix extension of the vector product (Sec. 2.1): y_i = a_i^T (+) w for row a_i of A.

    This is the numerator of the MAPI update, eq. (6), and Algorithm 1's product
    step.  A is read row by row, one vector product per row.
    """
    A = np.asarray(A, dtype=F64)
    w = np.asarray(w, dtype=F64)
    if A.ndim != 2 or A.shape[1] != w.shape[0]:
        raise ValueError(f"shape mismatch: A {A.shape}, w {w.shape}")
    y = np.empty(A.shape[0], dtype=F64)
    for i in range(A.shape[0]):
        y[i] = vec_product(A[i], w, op)
    return y


def normalize_l2(w):
    """The optional last step of Algorithm 1: w / ||w||_2."""
    w = np.asarray(w, dtype=F64)
    nrm = np.sqrt(np.sum(w * w))
    if not np.isfinite(nrm) or nrm == 0.0:
        raise OracleDegenerate("zero or non-finite l2 norm")
    return w / nrm


@dataclass
class IterResult:
    w: np.ndarray                     # final iterate (after the optional l2 step)
    iters: int                        # iterations run
    converged: bool                   # residual < tol was reached
    residuals: list = field(default_factory=list)   # ||w_t - w_{t-1}||_1 per iteration
    norms: list = field(default_factory=list)       # normaliser of each iteration


def _power_loop(step, w0, T, tol, norm):
    w = np.asarray(w0, dtype=F64).copy()
    res = IterResult(w=w, iters=0, converged=False)
    for _ in range(int(T)):
        y = step(w)
        if norm == "l1":
            nu = float(np.sum(np.abs(y)))
        elif norm == "l2":
            nu = float(np.sqrt(np.sum(y * y)))
        else:
            raise ValueError(norm)
        if not np.isfinite(nu) or nu == 0.0:
            raise OracleDegenerate(f"normaliser {nu!r} at iteration {res.iters + 1}")
        w_new = y / nu
        r = float(np.sum(np.abs(w_new - w)))
        w = w_new
        res.iters += 1
        res.norms.append(nu)
        res.residuals.append(r)
        if r < tol:
            res.converged = True
            break
    res.w = w
    return res


def mapi(A, w0, T, tol=0.0, op="min1", final_l2=False):
    """Multiplication-avoiding power iteration, eq. (6) and Algorithm 1.

    w0 is used exactly as given (the product is not homogeneous in w alone, so
    its scale matters).  Each of at most T iterations forms y = A (+) w and sets
    w = y / ||y||_1; iteration stops early once ||w_t - w_{t-1}||_1 < tol.  With
    ``final_l2`` the result is divided by its l2 norm (Algorithm 1, last step).
    """
    A = np.asarray(A, dtype=F64)
    res = _power_loop(lambda w: mavp(A, w, op), w0, T, tol, "l1")
    if final_l2:
        res.w = normalize_l2(res.w)
    return res


def rpi(A, b0, T, tol=0.0, norm="l2", final_l2=False):
    """Regular power iteration, eq. (1): b <- A b / ||A b||.

    ``norm`` is "l2" as eq. (1) states; PageRank uses the l1 normaliser, which
    leaves the direction unchanged.  The residual is ||b_t - b_{t-1}||_1.
    """
    A = np.asarray(A, dtype=F64)
    res = _power_loop(lambda b: A @ b, b0, T, tol, norm)
    if final_l2:
        res.w = normalize_l2(res.w)
    return res


def hybrid(A, w0, T_mapi, T_rpi, tol_mapi=0.0, tol_rpi=0.0, op="min1", final_l2=False):
    """MAPI, then RPI started from its result (Sec. 3.2, end of the comparison with
    stochastic PCA: to drive 1 - cos^2 to the top eigenvector towards zero, optimise
    with MAPI first and switch to RPI).  The MAPI result is divided by its l2 norm
    (Algorithm 1, last step) before it seeds eq. (1).  Returns (mapi result, rpi result).
    """
    m = mapi(A, w0, T_mapi, tol_mapi, op=op, final_l2=True)
    r = rpi(A, m.w, T_rpi, tol_rpi, final_l2=final_l2)
    return m, r


def ranks(w):
    """1-based indices of w ordered from its largest entry to its smallest.

    This is how the paper reports the ranks of its vectors (Sec. 3.2, Sec. 3.3).
    Ties go to the lower index.
    """
    w = np.asarray(w, dtype=F64)
    return [int(i) + 1 for i in np.argsort(-w, kind="stable")]
