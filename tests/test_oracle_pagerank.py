"""Pins of the oracle's PageRank forms (no GPU)."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth


def _graph(n, seed):
    g = synth.powerlaw_graph(n, seed)
    return g["n"], g["row_ptr"], g["col"], g["val"]


def test_dense_G_is_column_stochastic():
    n, rp, col, val = _graph(300, 1)
    G = oracle.dense_G(n, rp, col, val, 0.85)
    np.testing.assert_allclose(G.sum(axis=0), 1.0, rtol=1e-6)   # val is float32
    assert (G > 0).all()


def test_pagerank_rpi_matches_linear_solve():
    # Power iteration on G converges to the PageRank vector, which also solves
    # (I - alpha H~) x = (1 - alpha)/N 1 when sum(x) = 1.
    g = synth.powerlaw_graph(256, 2)
    n, rp, col = g["n"], g["row_ptr"], g["col"]
    val = 1.0 / g["outdeg"][col].astype(np.float64)     # exactly column-stochastic in float64
    alpha = 0.85
    G = oracle.dense_G(n, rp, col, val, alpha)
    Ht = (G - (1 - alpha) / n) / alpha
    x = scipy.linalg.solve(np.eye(n) - alpha * Ht, np.full(n, (1 - alpha) / n))
    x /= x.sum()
    w0 = synth.uniform_start(n)
    for form in ("dense", "csr"):
        r = oracle.pagerank(n, rp, col, val, alpha, "rpi", w0, T=300, tol=1e-15, form=form)
        np.testing.assert_allclose(r.w, x, rtol=1e-10, atol=1e-14)


def test_csr_split_equals_dense_product_on_4096_nodes():
    n, rp, col, val = _graph(4096, 3)
    G = oracle.dense_G(n, rp, col, val, 0.85)
    rng = np.random.default_rng(4)
    for w in (rng.standard_normal(n) / n, synth.uniform_start(n) * (1 + 0.1 * rng.uniform(size=n))):
        yd = oracle.pagerank_mavp_dense(G, w)
        yc = oracle.pagerank_mavp_csr(n, rp, col, val, 0.85, w)
        assert np.max(np.abs(yd - yc)) <= 1e-13 * np.max(np.abs(yd))


def test_csr_split_handles_explicit_dangling_nodes():
    # node 3 has no out-link; node 2 has no in-link
    g = synth.tiny_graph([(0, 1), (1, 0), (2, 0), (2, 1), (0, 3)], 4)
    n = 4
    mask = oracle.dangling_mask(n, g["col"])
    assert mask.tolist() == [False, False, False, True]
    G = oracle.dense_G(n, g["row_ptr"], g["col"], g["val"], 0.85)
    np.testing.assert_allclose(G[:, 3], 0.25)
    w = np.array([0.4, -0.1, 0.3, 0.2])
    np.testing.assert_allclose(oracle.pagerank_mavp_csr(n, g["row_ptr"], g["col"], g["val"], 0.85, w),
                               oracle.pagerank_mavp_dense(G, w), rtol=1e-14, atol=1e-16)


def test_mapi_pagerank_forms_agree():
    n, rp, col, val = _graph(512, 5)
    w0 = synth.uniform_start(n)
    rd = oracle.pagerank(n, rp, col, val, 0.85, "mapi", w0, T=6, form="dense")
    rc = oracle.pagerank(n, rp, col, val, 0.85, "mapi", w0, T=6, form="csr")
    np.testing.assert_allclose(rc.w, rd.w, rtol=1e-12)
    assert np.abs(rc.w).sum() == pytest.approx(1.0, rel=1e-14)
