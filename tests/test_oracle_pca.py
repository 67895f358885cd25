"""Pins of the oracle's covariance, min-covariance, deflation and top-k PCA (no GPU)."""
import numpy as np
import pytest

import oracle
import synth


def test_mingram_diagonal_is_scaled_l1_norm_and_symmetric():
    X = synth.pca_data(24, 300, seed=1)
    scale = 1.0 / 300
    A = oracle.mingram(X, scale)
    np.testing.assert_allclose(np.diag(A), scale * np.abs(X.astype(np.float64)).sum(axis=1), rtol=1e-14)
    np.testing.assert_array_equal(A, A.T)


def test_mingram_of_unit_modulus_data_is_covariance():
    # every |X_ik| = c: min1(a, b) = c sign(a) sign(b) = a b / c, so A = scale X X^T / c
    rng = np.random.default_rng(2)
    c = 0.75
    X = rng.choice([-c, c], size=(17, 101))
    A = oracle.mingram(X, 0.5)
    np.testing.assert_allclose(A, 0.5 * (X @ X.T) / c, rtol=1e-15, atol=1e-15)


def test_mingram_entry_agrees_with_full():
    X = synth.pca_data(12, 97, seed=3)
    A = oracle.mingram(X, 1 / 97)
    for i, j in [(0, 0), (3, 7), (11, 2)]:
        assert oracle.mingram_entry(X, i, j, 1 / 97) == pytest.approx(A[i, j], rel=1e-14)


def test_min2_gram_nonnegative():
    X = synth.pca_data(10, 50, seed=4)
    assert (oracle.mingram(X, 0.02, op="min2") >= 0).all()


def test_deflate_projection_annihilates_P():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((20, 20))
    P, _ = np.linalg.qr(rng.standard_normal((20, 3)))
    Ad = oracle.deflate_projection(A, P)
    assert np.max(np.abs(P.T @ Ad)) < 1e-13


def test_pca_topk_rpi_matches_eigh():
    A, Q, d = synth.planted_symmetric(64, [0.2, 0.2, 0.2, 0.15], seed=6)
    A = A.astype(np.float64)
    lam, V = np.linalg.eigh(A)
    W0 = synth.start_vectors(64, 4, seed=7)
    P, res = oracle.pca_topk(np.zeros((64, 1)), 4, W0, method="rpi", T=400, A=A)
    np.testing.assert_allclose(P.T @ P, np.eye(4), atol=1e-12)
    for i in range(4):
        cos = abs(np.dot(P[:, i], V[:, -1 - i]))
        assert cos > 1 - 1e-10, (i, cos)


def test_pca_topk_mapi_orthonormal_and_first_vector_is_mapi():
    X = synth.pca_data(32, 400, seed=8)
    W0 = synth.start_vectors(32, 3, seed=9)
    P, res = oracle.pca_topk(X, 3, W0, method="mapi", T=50)
    np.testing.assert_allclose(P.T @ P, np.eye(3), atol=1e-12)
    A = oracle.mingram(X, 1 / 400)
    r = oracle.mapi(A, W0[:, 0], 50)
    np.testing.assert_allclose(P[:, 0], r.w / np.linalg.norm(r.w), rtol=1e-12)
