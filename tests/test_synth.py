"""Seeded input generators: determinism and the structure of the synthetic workloads (no GPU)."""
import numpy as np

import synth


def test_generators_are_deterministic():
    a = synth.dense_cov(32, 64, seed=3)
    b = synth.dense_cov(32, 64, seed=3)
    assert a.tobytes() == b.tobytes()
    assert synth.dense_cov(32, 64, seed=4).tobytes() != a.tobytes()
    g1 = synth.powerlaw_graph(1000, seed=5)
    g2 = synth.powerlaw_graph(1000, seed=5)
    for k in ("row_ptr", "col", "val"):
        assert g1[k].tobytes() == g2[k].tobytes()
    assert synth.pca_data(8, 50, 6).tobytes() == synth.pca_data(8, 50, 6).tobytes()


def test_dense_cov_is_symmetric_psd():
    C = synth.dense_cov(40, 200, seed=1).astype(np.float64)
    np.testing.assert_allclose(C, C.T, rtol=1e-6, atol=1e-7)
    assert np.linalg.eigvalsh(C).min() > -1e-5


def test_start_vector_unit_l2():
    w = synth.start_vector(1000, 2).astype(np.float64)
    assert abs(np.linalg.norm(w) - 1) < 1e-6


def test_powerlaw_graph_structure():
    n = 1 << 14
    g = synth.powerlaw_graph(n, seed=7)
    rp, col, val, outdeg = g["row_ptr"], g["col"], g["val"], g["outdeg"]
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    dst = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(dst == col)                              # no self-links
    key = dst.astype(np.int64) * n + col
    assert np.unique(key).size == key.size                     # duplicates merged
    sums = np.bincount(col, weights=val.astype(np.float64), minlength=n)
    live = outdeg > 0
    np.testing.assert_allclose(sums[live], 1.0, rtol=1e-6)     # column-stochastic
    dang = (~live).mean()
    assert 0.04 < dang < 0.08                                  # seeded 5 % plus Zipf zeros
    assert 13 < col.size / n < 17                              # mean out-degree about 16 * 0.95
    assert outdeg.max() > 200                                  # heavy tail


def test_dyadic_values():
    A = synth.dyadic_matrix(10, 20, seed=8)
    assert np.all((A * 8) == np.round(A * 8)) and np.abs(A).max() <= 2


def test_laplace_from_uniform_is_finite_and_laplace():
    import torch
    # r = 0 is a value float32 uniform generators return; it must not give an infinity
    r = torch.tensor([0.0, 0.25, 0.5, 0.75, 1.0 - 2.0 ** -24], dtype=torch.float32)
    x = synth.laplace_from_uniform(r, 10.0)
    assert torch.isfinite(x).all()
    assert abs(float(x[0]) - 10.0 * np.log(2.0 ** -24)) < 1e-3   # clamped end: u = -1/2 + 2^-25
    assert float(x[2]) == 0.0
    # the inverse CDF: P(X <= x) = 1/2 exp(x / b) for x < 0, so r = 1/4 maps to b log(1/2)
    assert abs(float(x[1]) - 10.0 * np.log(0.5)) < 1e-5 and abs(float(x[3]) + 10.0 * np.log(0.5)) < 1e-5
    # moments of a large sample: mean 0, E|X| = b
    g = torch.Generator().manual_seed(3)
    s = synth.laplace_from_uniform(torch.rand(200000, generator=g), 2.0).double()
    assert abs(float(s.mean())) < 0.03 and abs(float(s.abs().mean()) - 2.0) < 0.03


def test_sec32_data_has_the_stated_spectrum():
    X, v1 = synth.sec32_data(5000, 10, seed=2)
    C = X.astype(np.float64).T @ X.astype(np.float64) / 5000
    lam, V = np.linalg.eigh(C)
    np.testing.assert_allclose(lam[::-1], [1.0] + [0.9] * 9, atol=1e-5)
    assert abs(abs(V[:, -1] @ v1) - 1.0) < 1e-9


def test_minibatch_indices_range_and_shape():
    b = synth.minibatch_indices(3, 4, 5, 17, seed=1)
    assert b.shape == (3, 4, 5) and b.dtype == np.int32
    assert b.min() >= 0 and b.max() < 17


def test_generated_start_is_the_generated_problems_start():
    # the start vector alone (the seeded PCA starts) equals the one generated_dense returns,
    # has entries +-fl32(1/sqrt(n)) and unit l2 norm up to rounding, and differs between seeds
    for n, seed in ((1, 0), (7, 3), (300, 12)):
        _, w0 = synth.generated_dense(n, seed)
        ws = synth.generated_start(n, seed)
        np.testing.assert_array_equal(ws, w0)
        assert set(np.abs(ws).tolist()) == {float(np.float32(1.0 / np.sqrt(n)))}
        assert abs(float(np.linalg.norm(ws.astype(np.float64))) - 1.0) < 1e-6
    assert not np.array_equal(synth.generated_start(300, 0), synth.generated_start(300, 1))
