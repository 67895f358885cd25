"""Pins of the factored-operator oracle (oracle/factored.py; not a method of the paper): the
sign-matrix reduction against numpy matmul and numpy.linalg.eigh, exact rational brute force
on tiny dyadic matrices, and the difference from Alg. 1 on eq. (5)'s min-covariance."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

REL = 1e-12


def sgn(x):
    return (x > 0) - (x < 0)


def min1_exact(a, b):
    return sgn(a) * sgn(b) * min(abs(a), abs(b))


def min2_exact(a, b):
    return min(abs(a), abs(b)) if sgn(a) == sgn(b) else Fr(0)


def factored_exact(X, w, scale, term):
    """z_k = sum_i term(X_ik, w_i); y_i = scale * sum_k term(X_ik, z_k), in rationals."""
    D, N = len(X), len(X[0])
    z = [sum((term(X[i][k], w[i]) for i in range(D)), Fr(0)) for k in range(N)]
    return [scale * sum((term(X[i][k], z[k]) for k in range(N)), Fr(0)) for i in range(D)]


def _sign_dominated(rng, D, N):
    X = rng.uniform(1.0, 3.0, size=(D, N)) * np.where(rng.uniform(size=(D, N)) < 0.6, 1.0, -1.0)
    return X


def test_one_step_is_the_sign_matrix_product():
    # |X_ik| >= 1 and ||w||_1 <= 1: z = S^T w exactly (|w_i| <= 1 <= |X_ik|), |z_k| <= 1, and
    # y = scale * S z; a transposed first product (X (+) w with w of length N) cannot even be formed
    rng = np.random.default_rng(3)
    D, N = 12, 30
    X = _sign_dominated(rng, D, N)
    S = np.sign(X)
    w = rng.uniform(-1, 1, D)
    w /= np.abs(w).sum()
    got = oracle.factored_product(X, w, scale=1.0 / N)
    want = (1.0 / N) * (S @ (S.T @ w))
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)
    # the min2 form reduces to the positive parts: 1(sign X = sign w) min(|X|, |w|) = [S > 0] w+ + [S < 0] w-
    got2 = oracle.factored_product(X, w, op="min2")
    P, M = (S > 0).astype(float), (S < 0).astype(float)
    z2 = P.T @ np.maximum(w, 0) - M.T @ np.minimum(w, 0)
    want2 = P @ np.maximum(z2, 0) - M @ np.minimum(z2, 0)
    np.testing.assert_allclose(got2, want2, rtol=1e-13, atol=1e-15)


def test_iteration_reaches_the_top_eigenvector_of_the_sign_gram():
    rng = np.random.default_rng(4)
    D, N = 10, 200
    # a dominant direction: rows share the sign pattern of a planted vector on most samples
    base = np.where(rng.uniform(size=N) < 0.5, 1.0, -1.0)
    X = _sign_dominated(rng, D, N)
    flip = rng.uniform(size=(D, N)) < 0.8
    X = np.where(flip, np.abs(X) * base[None, :], X)
    S = np.sign(X)
    vals, vecs = np.linalg.eigh(S @ S.T)
    top = vecs[:, -1]
    assert vals[-1] > 1.5 * vals[-2]
    w0 = np.full(D, 1.0 / D)
    res = oracle.factored_mapi(X, w0, 200, tol=1e-15)
    cos = abs(np.dot(res.w, top)) / np.linalg.norm(res.w)
    assert cos > 1 - 1e-10
    assert np.abs(res.w).sum() == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("op,term", [("min1", min1_exact), ("min2", min2_exact)])
def test_factored_iterates_are_exact_on_dyadic_matrices(op, term):
    rng = np.random.default_rng(20211023)
    for c in range(24):
        D, N = 1 + c % 6, 1 + (c * 5) % 6
        X = rng.integers(-16, 17, size=(D, N)) / 8.0
        w0 = rng.integers(-16, 17, size=D) / 8.0
        if not w0.any():
            w0[0] = 0.5
        scale = Fr(1, N)
        Xf = [[Fr(float(v)) for v in row] for row in X]
        w = [Fr(float(v)) for v in w0]
        y = factored_exact(Xf, w, scale, term)
        got = oracle.factored_product(X, w0, 1.0 / N, op)
        s = float(sum(abs(v) for v in y)) + 1e-300
        assert all(abs(float(a) - float(b)) <= REL * s for a, b in zip(got, y))
        # iterates, normalisers and l1 residuals of up to 4 steps
        ws, nus, rs = [], [], []
        for _ in range(4):
            y = factored_exact(Xf, w, scale, term)
            nu = sum((abs(v) for v in y), Fr(0))
            if nu == 0:
                break
            wn = [v / nu for v in y]
            rs.append(sum((abs(a - b) for a, b in zip(wn, w)), Fr(0)))
            nus.append(nu)
            ws.append(wn)
            w = wn
        if not nus:
            with pytest.raises(oracle.OracleDegenerate):
                oracle.factored_mapi(X, w0, 1, scale=1.0 / N, op=op)
            continue
        res = oracle.factored_mapi(X, w0, len(nus), scale=1.0 / N, op=op)
        assert res.iters == len(nus)
        for a, b in zip(res.norms, nus):
            assert abs(a - float(b)) <= REL * float(b)
        for a, b in zip(res.residuals, rs):
            assert abs(a - float(b)) <= REL * 2.0
        assert np.all(np.abs(res.w - np.array([float(v) for v in ws[-1]])) <= REL)


def test_factored_operator_is_not_alg1_on_the_min_covariance():
    # (+) is not associative: the factored iteration and Alg. 1 on A = (1/N) X (+) X^T part ways
    rng = np.random.default_rng(5)
    D, N = 16, 64
    X = rng.standard_normal((D, N))
    w0 = rng.uniform(-1, 1, D)
    w0 /= np.abs(w0).sum()
    a = oracle.factored_mapi(X, w0, 5, scale=1.0 / N).w
    b = oracle.mapi(oracle.mingram(X, 1.0 / N), w0, 5).w
    assert np.abs(a - b).sum() > 1e-3
