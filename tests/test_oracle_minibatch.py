"""Pins of the mini-batch MAPI oracle (Algorithm 3)."""
import numpy as np
import pytest

import oracle
import synth


def test_full_batches_without_momentum_are_algorithm_1():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((9, 40))
    w0 = synth.start_vector(9, 4).astype(np.float64)
    T = 12
    batches = np.tile(np.arange(40), (T, 1))
    r = oracle.minibatch_mapi(X, batches, 0.0, w0)
    ref = oracle.mapi(oracle.mingram(X, 1.0 / 40), w0, T)
    assert r.iters == T
    np.testing.assert_array_equal(r.w, ref.w)


@pytest.mark.parametrize("beta", [0.0, 0.15, 0.6])
def test_sign_aligned_data_follow_the_momentum_recurrence(beta):
    # every sample shares the sign pattern sigma and has entries of modulus >= 1, so each batch
    # matrix has |A_kl| >= 1 and A (+) w = sigma (sigma^T w) while ||w||_1 = 1
    rng = np.random.default_rng(5)
    D, N, s, T = 7, 30, 4, 9
    sigma = np.where(rng.uniform(size=D) < 0.5, -1.0, 1.0)
    X = sigma[:, None] * (1.0 + rng.uniform(size=(D, N)) * 3.0)
    batches = rng.integers(0, N, size=(T, s))
    w0 = synth.start_vector(D, 6).astype(np.float64)
    w0 = w0 / np.sum(np.abs(w0))
    r = oracle.minibatch_mapi(X, batches, beta, w0)
    S = np.outer(sigma, sigma)                    # sign of every batch matrix
    w_prev, w = np.zeros(D), w0.copy()
    for _ in range(T):
        w_next = S @ w - beta * w_prev
        nu = np.sum(np.abs(w_next))
        w_prev, w = w / nu, w_next / nu
    np.testing.assert_allclose(r.w, w, rtol=0, atol=1e-14)


def test_dot_form_is_the_stochastic_power_method():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((6, 25))
    batches = rng.integers(0, 25, size=(5, 3))
    w0 = synth.start_vector(6, 9).astype(np.float64)
    r = oracle.minibatch_mapi(X, batches, 0.1, w0, op="dot")
    w_prev, w = np.zeros(6), w0.copy()
    for B in batches:
        A = X[:, B] @ X[:, B].T / len(B)
        w_next = A @ w - 0.1 * w_prev
        nu = np.sum(np.abs(w_next))
        w_prev, w = w / nu, w_next / nu
    np.testing.assert_allclose(r.w, w, rtol=1e-13, atol=0)


def test_degenerate_batch_raises():
    X = np.zeros((4, 10))
    with pytest.raises(oracle.OracleDegenerate):
        oracle.minibatch_mapi(X, np.zeros((2, 3), dtype=int), 0.0, np.ones(4) / 4)
