"""Pins of the image-reconstruction oracle (Algorithm 2)."""
import numpy as np
import pytest

import oracle
import synth


def test_min_outer_identities():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((30, 2))
    M = oracle.min_outer(W)
    np.testing.assert_array_equal(M, M.T)
    np.testing.assert_allclose(np.diag(M), np.abs(W).sum(axis=1), rtol=0, atol=1e-15)
    # columns of constant modulus: min(|a|, |b|) = c, so the extension is c sign(W) sign(W)^T
    S = np.where(rng.uniform(size=(30, 2)) < 0.5, -1.0, 1.0)
    Wc = S * np.array([0.3, 0.7])[None, :]
    np.testing.assert_allclose(oracle.min_outer(Wc), (S * [0.3, 0.7]) @ S.T, rtol=0, atol=1e-15)


def test_rpi_reconstruction_is_the_top2_projection():
    clean, V = synth.occluded_images(16, 10, seed=3)
    w0 = synth.start_vector(256, 4).astype(np.float64)
    R, W, (r1, r2) = oracle.image_reconstruct(V, 3000, w0, method="rpi", tol=1e-15)
    Vd = V.astype(np.float64)
    m = Vd.mean(axis=1)
    C = np.cov(Vd)                                    # (1/(N-1)) centred, numpy's definition
    lam, E = np.linalg.eigh(C)
    top = E[:, -2:]
    assert np.linalg.norm(W.T @ W - np.eye(2)) < 1e-6  # RPI vectors are orthonormal here
    np.testing.assert_allclose(W @ W.T, top @ top.T, rtol=0, atol=1e-6)
    np.testing.assert_allclose(R, top @ (top.T @ (Vd - m[:, None])) + m[:, None], rtol=0, atol=1e-6)


def test_mapi_reconstruction_shapes_and_psnr_is_finite():
    clean, V = synth.occluded_images(16, 10, seed=5)
    w0 = synth.start_vector(256, 6).astype(np.float64)
    R, W, _ = oracle.image_reconstruct(V, 40, w0)
    assert R.shape == (256, 10) and W.shape == (256, 2)
    np.testing.assert_allclose(np.abs(W).sum(axis=0), 1.0, rtol=1e-14)    # Algorithm 1's l1 normalisation
    p = [oracle.psnr(R[:, i], clean) for i in range(10)]
    assert all(np.isfinite(p))


def test_min_outer_of_a_flat_l1_unit_vector_reproduces_it():
    # the reason for l1 units: for |w_j| = 1/P, (w (+) w^T) w = w exactly (w (+) w = ||w||_1 = 1)
    P = 50
    s = np.where(np.random.default_rng(2).uniform(size=P) < 0.5, -1.0, 1.0)
    w = s / P
    np.testing.assert_allclose(oracle.min_outer(w) @ w, w, rtol=0, atol=1e-16)


def test_occluded_images_structure():
    clean, V = synth.occluded_images(32, 6, seed=7)
    assert clean.min() >= 0 and clean.max() <= 1 and V.shape == (1024, 6)
    for i in range(6):
        diff = (V[:, i] != clean).reshape(32, 32)
        bad = [diff[r * 8:(r + 1) * 8, c * 8:(c + 1) * 8].any() for r in range(4) for c in range(4)]
        assert sum(bad) == 3


def _flat(rng, P, c):
    s = np.where(rng.uniform(size=P) < 0.5, -1.0, 1.0)
    return s, c * s


def test_minouter_deflation_multiplies_from_the_left():
    # Alg. 2 deflation: for w = c s (constant modulus), w (+) w^T = c s s^T, so the step is
    # C - c s (s^T C); the right-hand product C - C (c s s^T) differs for a generic C
    rng = np.random.default_rng(11)
    P = 40
    X = rng.standard_normal((P, 7))
    C = oracle.mingram(X, 1.0 / 6)
    s, w = _flat(rng, P, 1.0 / P)
    got = oracle.minouter_deflate(C, w)
    want = C - (1.0 / P) * np.outer(s, s @ C)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
    wrong = C - (1.0 / P) * np.outer(C @ s, s)
    assert np.max(np.abs(wrong - want)) > 1e-3


def test_minouter_reconstruction_of_flat_vectors():
    # Alg. 2 reconstruction: with W = [c1 s1, c2 s2], W (+) W^T = c1 s1 s1^T + c2 s2 s2^T
    rng = np.random.default_rng(12)
    P, N = 36, 5
    s1, w1 = _flat(rng, P, 1.0 / P)
    s2, w2 = _flat(rng, P, 0.5 / P)
    Vc = rng.standard_normal((P, N))
    m = rng.uniform(size=P)
    R = oracle.minouter_reconstruct(np.stack([w1, w2], axis=1), Vc, m)
    want = (1.0 / P) * np.outer(s1, s1 @ Vc) + (0.5 / P) * np.outer(s2, s2 @ Vc) + m[:, None]
    np.testing.assert_allclose(R, want, rtol=0, atol=1e-14)
    # a single column is not the same as the pair (the sum over the columns of W is taken)
    R1 = oracle.minouter_reconstruct(w1[:, None], Vc, m)
    assert np.max(np.abs(R1 - want)) > 1e-3


def test_mapi_reconstruction_is_the_composition_of_the_pinned_steps():
    clean, V = synth.occluded_images(16, 10, seed=5)
    w0 = synth.start_vector(256, 6).astype(np.float64)
    R, W, (r1, r2) = oracle.image_reconstruct(V, 25, w0)
    Vd = V.astype(np.float64)
    m = Vd.mean(axis=1)
    Vc = Vd - m[:, None]
    C = oracle.mingram(Vc, 1.0 / 9)                       # eq. (5) with Alg. 2's 1/(N-1)
    a1 = oracle.mapi(C, w0, 25)
    np.testing.assert_array_equal(W[:, 0], a1.w)
    a2 = oracle.mapi(oracle.minouter_deflate(C, a1.w), w0, 25)
    np.testing.assert_array_equal(W[:, 1], a2.w)
    np.testing.assert_array_equal(R, oracle.minouter_reconstruct(np.stack([a1.w, a2.w], axis=1), Vc, m))


def test_min2_minouter_deflation_and_reconstruction_of_flat_vectors():
    # min2 (eq. 4): for w = c s, the term 1(s_i = s_j) min(c, c) gives w (+) w^T = c (1 1^T + s s^T) / 2,
    # so Alg. 2's deflation is C - (c/2)(1 (1^T C) + s (s^T C)) and the reconstruction of
    # W = [c1 s1, c2 s2] is sum_k (c_k/2)(1 (1^T Vc) + s_k (s_k^T Vc)) + m (numpy, fixed product order)
    rng = np.random.default_rng(13)
    P, N = 40, 6
    X = rng.standard_normal((P, 7))
    C = oracle.mingram(X, 1.0 / 6, "min2")
    s, w = _flat(rng, P, 1.0 / P)
    one = np.ones(P)
    got = oracle.minouter_deflate(C, w, "min2")
    want = C - (0.5 / P) * (np.outer(one, one @ C) + np.outer(s, s @ C))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
    wrong = C - (0.5 / P) * (np.outer(C @ one, one) + np.outer(C @ s, s))
    assert np.max(np.abs(wrong - want)) > 1e-3
    s2, w2 = _flat(rng, P, 0.5 / P)
    Vc = rng.standard_normal((P, N))
    m = rng.uniform(size=P)
    R = oracle.minouter_reconstruct(np.stack([w, w2], axis=1), Vc, m, "min2")
    want = ((0.5 / P) * (np.outer(one, one @ Vc) + np.outer(s, s @ Vc))
            + (0.25 / P) * (np.outer(one, one @ Vc) + np.outer(s2, s2 @ Vc)) + m[:, None])
    np.testing.assert_allclose(R, want, rtol=0, atol=1e-14)


def test_min2_reconstruction_is_the_composition_of_the_pinned_steps():
    clean, V = synth.occluded_images(16, 10, seed=7)
    w0 = synth.start_vector(256, 8).astype(np.float64)
    R, W, _ = oracle.image_reconstruct(V, 20, w0, op="min2")
    Vd = V.astype(np.float64)
    m = Vd.mean(axis=1)
    Vc = Vd - m[:, None]
    C = oracle.mingram(Vc, 1.0 / 9, "min2")
    a1 = oracle.mapi(C, w0, 20, op="min2")
    np.testing.assert_array_equal(W[:, 0], a1.w)
    a2 = oracle.mapi(oracle.minouter_deflate(C, a1.w, "min2"), w0, 20, op="min2")
    np.testing.assert_array_equal(W[:, 1], a2.w)
    np.testing.assert_array_equal(R, oracle.minouter_reconstruct(np.stack([a1.w, a2.w], axis=1), Vc, m, "min2"))
