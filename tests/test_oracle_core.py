"""Pins of the oracle's operators, MAVP product, MAPI and RPI loops (no GPU).

Each test checks the oracle against something fixed outside it: an identity of
the operator, a closed form, a library eigen-solver or values printed in the
paper.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- operators
def test_min1_min2_truth_table():
    # eq. (3) and eq. (4) worked by hand on scalar pairs
    cases = [  # a, b, min1, min2
        (3.0, -2.0, -2.0, 0.0),
        (-1.0, -5.0, 1.0, 1.0),
        (2.0, 3.0, 2.0, 2.0),
        (-4.0, 0.5, -0.5, 0.0),
        (0.0, 5.0, 0.0, 0.0),
        (7.0, 0.0, 0.0, 0.0),
    ]
    for a, b, m1, m2 in cases:
        assert oracle.term_min1(a, b) == m1
        assert oracle.term_min2(a, b) == m2


@pytest.mark.parametrize("op", ["min1", "min2"])
def test_l1_identity(op):
    # x (+) x = ||x||_1 (Sec. 2.1, text after eq. 4)
    rng = np.random.default_rng(1)
    for n in (1, 7, 64, 1000):
        x = rng.standard_normal(n) * rng.uniform(0.01, 100)
        assert oracle.vec_product(x, x, op) == pytest.approx(np.abs(x).sum(), rel=1e-15)


def test_min1_symmetry_oddness_homogeneity():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(513)
    b = rng.standard_normal(513) * 3
    p = oracle.vec_product(a, b)
    assert oracle.vec_product(b, a) == p                      # symmetric
    assert oracle.vec_product(-a, b) == -p                    # odd in each argument
    assert oracle.vec_product(a, -b) == -p
    for lam in (0.25, 4.0, 1024.0):                           # exact powers of two
        assert oracle.vec_product(lam * a, lam * b) == lam * p
    assert oracle.vec_product(3.7 * a, 3.7 * b) == pytest.approx(3.7 * p, rel=1e-14)
    # not homogeneous in one argument alone: the scale of w0 matters for MAPI
    assert abs(oracle.vec_product(3 * a, b) - 3 * p) > 1e-3 * abs(p)


def test_min1_from_min2_and_bounds():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(300)
    b = rng.standard_normal(300)
    np.testing.assert_array_equal(oracle.term_min1(a, b),
                                  oracle.term_min2(a, b) - oracle.term_min2(-a, b))
    p = oracle.vec_product(a, b)
    bound = np.minimum(np.abs(a), np.abs(b)).sum()
    assert abs(p) <= bound <= min(np.abs(a).sum(), np.abs(b).sum())
    perm = rng.permutation(300)
    assert oracle.vec_product(a[perm], b[perm]) == pytest.approx(p, rel=1e-14, abs=1e-14)
    assert oracle.vec_product(a, b, "min2") >= 0.0            # min2 never negative


def test_diamond_forms_agree():
    # eq. (7): sign(a) b + a sign(b) equals sign(a b)(|a| + |b|) for reals
    rng = np.random.default_rng(4)
    a = rng.standard_normal(100)
    b = rng.standard_normal(100)
    np.testing.assert_allclose(oracle.term_diamond(a, b),
                               np.sign(a * b) * (np.abs(a) + np.abs(b)), rtol=1e-15)


# ---------------------------------------------------------------- MAVP product
def test_mavp_sign_reduction_fixes_orientation():
    # If |A_ij| >= 1 >= |w_j| every term is sign(A_ij) w_j, so A (+) w = sign(A) @ w.
    rng = np.random.default_rng(5)
    m, n = 37, 53
    A = rng.choice([-1.0, 1.0], size=(m, n)) * rng.uniform(1.0, 3.0, size=(m, n))
    w = rng.uniform(-1.0, 1.0, size=n)
    y = oracle.mavp(A, w)
    np.testing.assert_allclose(y, np.sign(A) @ w, rtol=1e-13, atol=1e-13)
    B = rng.choice([-1.0, 1.0], size=(n, n)) * rng.uniform(1.0, 3.0, size=(n, n))
    yb = oracle.mavp(B, w)
    assert np.max(np.abs(yb - np.sign(B).T @ w)) > 1e-3      # the transpose would be caught


def test_mavp_rejects_shape_mismatch():
    with pytest.raises(ValueError):
        oracle.mavp(np.ones((3, 4)), np.ones(3))


# ---------------------------------------------------------------- MAPI (Algorithm 1)
def test_mapi_iterates_have_unit_l1():
    # Sec. 2.2: the normalisation keeps ||w_t||_1 = 1
    A = synth.dense_cov(48, 200, seed=6).astype(np.float64)
    w0 = synth.start_vector(48, 7)
    for T in (1, 2, 5):
        r = oracle.mapi(A, w0, T)
        assert r.iters == T
        assert np.abs(r.w).sum() == pytest.approx(1.0, rel=1e-14)
        assert len(r.residuals) == T and len(r.norms) == T


def test_mapi_equals_l1_power_iteration_on_sign_matrix():
    # With |A_ij| >= 1 and ||w||_1 <= 1 every step is w <- S w / ||S w||_1, S = sign(A),
    # so MAPI converges to the dominant eigenvector of S (numpy.linalg.eigh).
    rng = np.random.default_rng(8)
    n = 64
    S = np.where(rng.uniform(size=(n, n)) < 0.8, 1.0, -1.0)
    S = np.triu(S) + np.triu(S, 1).T
    M = rng.uniform(1.0, 3.0, size=(n, n))
    A = S * (np.triu(M) + np.triu(M, 1).T)
    lam, V = np.linalg.eigh(S)
    assert lam[-1] > 2 * abs(lam[0])
    u = V[:, -1]
    r = oracle.mapi(A, synth.uniform_start(n), T=60)
    cos = abs(np.dot(r.w, u)) / np.linalg.norm(r.w)
    assert cos > 1 - 1e-12
    # each step is exactly the l1-normalised sign(A) product
    w1 = oracle.mapi(A, synth.uniform_start(n), T=1).w
    s = S @ synth.uniform_start(n).astype(np.float64)
    np.testing.assert_allclose(w1, s / np.abs(s).sum(), rtol=1e-13)


def test_mapi_constant_matrix_reaches_uniform_in_one_step():
    n = 33
    A = np.full((n, n), 0.7)
    w0 = synth.start_vector(n, 9)
    w0[0] = 0.9  # makes sum_j sign(w_j) min(0.7, |w_j|) positive
    assert oracle.vec_product(np.full(n, 0.7), w0) > 0
    r = oracle.mapi(A, w0, T=1)
    np.testing.assert_allclose(r.w, np.full(n, 1.0 / n), rtol=1e-14)


def test_proposition1_closed_form_in_two_iterations():
    # Proposition 1: for positive A and a positive start, the diamond iteration reaches
    # (1 + ||a_i||_1) / sum_j (1 + ||a_j||_1) at the second iteration and stays there.
    rng = np.random.default_rng(10)
    n = 20
    A = rng.uniform(0.1, 2.0, size=(n, n))
    w0 = rng.uniform(0.1, 1.0, size=n)
    row = 1.0 + np.abs(A).sum(axis=1)
    target = row / row.sum()
    r1 = oracle.mapi(A, w0, T=1, op="diamond")
    assert np.max(np.abs(r1.w - target)) > 1e-6
    for T in (2, 3, 6):
        r = oracle.mapi(A, w0, T=T, op="diamond")
        np.testing.assert_allclose(r.w, target, rtol=1e-13)


def test_mapi_tolerance_stops_and_reports():
    rng = np.random.default_rng(11)
    n = 30
    A = rng.uniform(0.01, 0.3, size=(n, n))
    A = (A + A.T) / 2
    w0 = synth.start_vector(n, 12)
    r = oracle.mapi(A, w0, T=500, tol=1e-12)
    assert r.converged and 3 < r.iters < 500 and r.residuals[-1] < 1e-12
    r2 = oracle.mapi(A, w0, T=3, tol=1e-12)
    assert not r2.converged and r2.iters == 3


def test_mapi_degenerate_raises():
    with pytest.raises(oracle.OracleDegenerate):
        oracle.mapi(np.zeros((4, 4)), np.ones(4) / 4, T=3)


def test_mapi_final_l2():
    A = synth.dense_cov(16, 64, seed=12).astype(np.float64)
    r = oracle.mapi(A, synth.start_vector(16, 13), T=10, final_l2=True)
    assert np.sqrt(np.sum(r.w ** 2)) == pytest.approx(1.0, rel=1e-14)


# ---------------------------------------------------------------- RPI (eq. 1)
def test_rpi_matches_eigh_on_planted_gap():
    A, Q, d = synth.planted_symmetric(80, [0.3], seed=14)
    A = A.astype(np.float64)
    lam, V = np.linalg.eigh(A)
    r = oracle.rpi(A, synth.start_vector(80, 15), T=300)
    cos = abs(np.dot(r.w, V[:, -1]))
    assert cos > 1 - 1e-12
    assert np.sqrt(np.sum(r.w ** 2)) == pytest.approx(1.0, rel=1e-14)
    assert r.norms[-1] == pytest.approx(lam[-1], rel=1e-10)


# ---------------------------------------------------------------- printed values
def test_ranks_match_paper_printed_lists():
    with open(os.path.join(GOLDEN, "paper_printed_vectors.json")) as f:
        g = json.load(f)
    for key, item in g.items():
        if key.startswith("_"):
            continue
        assert oracle.ranks(item["w"]) == item["ranks"], key


def test_printed_vectors_are_l2_normalised():
    # The printed final vectors went through Algorithm 1's optional l2 step: their
    # norms are 1 up to the three-decimal rounding of the print.
    with open(os.path.join(GOLDEN, "paper_printed_vectors.json")) as f:
        g = json.load(f)
    for key, item in g.items():
        if key.startswith("_"):
            continue
        w = np.array(item["w"])
        slack = 0.0005 * np.abs(w).sum() * 2 + 1e-3
        assert abs(np.linalg.norm(w) - 1.0) < slack, key


def test_hybrid_without_mapi_steps_is_rpi_from_the_start_direction():
    # zero MAPI iterations hand over w0 / ||w0||_2; eq. (1) is invariant to a positive scale of
    # its start, so the hybrid is RPI from w0 (the MAPI phase is then the identity)
    A, Q, d = synth.planted_symmetric(40, [0.3], seed=7)
    w0 = synth.start_vector(40, 8).astype(np.float64) * 3.7
    m, r = oracle.hybrid(A, w0, 0, 25)
    ref = oracle.rpi(A, w0, 25)
    assert m.iters == 0
    np.testing.assert_allclose(m.w, w0 / np.linalg.norm(w0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(r.w, ref.w, rtol=0, atol=1e-12)


def test_hybrid_hands_over_the_unit_l2_mapi_iterate_and_reaches_the_eigenvector():
    A, Q, d = synth.planted_symmetric(64, [0.2], seed=11)
    A = np.abs(A) + 0.05          # positive entries: min1 iterates keep the sign structure of eq. (1)
    lam, V = np.linalg.eigh(A.astype(np.float64))
    u = V[:, -1]
    w0 = np.abs(synth.start_vector(64, 12)).astype(np.float64)
    m, r0 = oracle.hybrid(A, w0, 30, 0)
    assert abs(np.linalg.norm(m.w) - 1.0) < 1e-15 and r0.iters == 0
    np.testing.assert_allclose(r0.w, m.w, rtol=0, atol=0)
    m, r = oracle.hybrid(A, w0, 30, 400, tol_rpi=1e-14)
    cos = abs(float(r.w @ u)) / np.linalg.norm(r.w)
    assert 1.0 - cos * cos < 1e-14      # float64 resolution of cos near 1
