"""GPU parity of MAPI and RPI PageRank (eq. 11) on CSR link matrices against the FP64 oracle."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from gpu_util import rel_l1, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5


def _dev(g):
    return (torch.from_numpy(g["row_ptr"]).cuda(), torch.from_numpy(g["col"]).cuda(),
            torch.from_numpy(g["val"]).cuda())


@pytest.mark.parametrize("method", ["mapi", "rpi"])
@pytest.mark.parametrize("T", [1, 5, 30])
def test_pagerank_4096_nodes_matches_dense_oracle(method, T):
    g = synth.powerlaw_graph(4096, seed=9)
    rp, col, val = _dev(g)
    w, info = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=T)
    assert info["iters"] == T
    ref = oracle.pagerank(4096, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(4096), T,
                          form="dense")
    wg = w.cpu().numpy()
    e, _ = report(f"pagerank {method} n=4096 T={T}", wg, ref.w)
    assert e <= TOL
    # the ranking signal sits in the deviation from uniform; report its error too
    report(f"pagerank {method} n=4096 T={T} deviation from 1/n", wg - 1 / 4096, ref.w - 1 / 4096)


def test_pagerank_rpi_reaches_linear_solve():
    g = synth.powerlaw_graph(1024, seed=10)
    n = 1024
    rp, col, val = _dev(g)
    # a float32 iterate of entries ~1/n changes by ~n ulp(1/n) ~ 1e-7 per step at its fixed point,
    # so the stop tolerance is set above that floor
    w, info = mp.mapi_pagerank(rp, col, val, 0.85, "rpi", max_iters=300, tol=2e-7)
    assert info["converged"]
    G = oracle.dense_G(n, g["row_ptr"], g["col"], g["val"], 0.85)
    Ht = (G - 0.15 / n) / 0.85
    x = scipy.linalg.solve(np.eye(n) - 0.85 * Ht, np.full(n, 0.15 / n))
    x /= x.sum()
    assert rel_l1(w.cpu().numpy(), x) <= TOL


def test_pagerank_tolerance_and_iteration_parity():
    g = synth.powerlaw_graph(3000, seed=11)
    rp, col, val = _dev(g)
    for method in ("mapi", "rpi"):
        w, info = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=200, tol=1e-7, check_every=4)
        assert info["converged"]
        ref = oracle.pagerank(3000, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(3000),
                              info["iters"])
        assert rel_l1(w.cpu().numpy(), ref.w) <= TOL
        print(f"[iters] {method}: gpu {info['iters']}", flush=True)


def test_pagerank_explicit_dangling_and_custom_start():
    g = synth.tiny_graph([(0, 1), (1, 0), (2, 0), (2, 1), (0, 3)], 4)
    rp, col, val = _dev(g)
    w0 = np.array([0.4, 0.1, 0.3, 0.2], np.float32)
    for method in ("mapi", "rpi"):
        w, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, w0=torch.from_numpy(w0).cuda(), max_iters=20,
                                final_l2=True)
        ref = oracle.pagerank(4, g["row_ptr"], g["col"], g["val"], 0.85, method, w0, 20, form="dense")
        r = ref.w / np.linalg.norm(ref.w)
        assert rel_l1(w.cpu().numpy(), r) <= TOL


def test_pagerank_graph_without_links():
    n = 100
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    val = torch.zeros(0, dtype=torch.float32, device="cuda")
    w, info = mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=3)
    np.testing.assert_allclose(w.cpu().numpy(), 1.0 / n, rtol=1e-6)


@pytest.mark.parametrize("bad", ["col_range", "row_ptr_order", "row_ptr_end"])
def test_invalid_csr_is_rejected(bad):
    g = synth.powerlaw_graph(500, seed=12)
    rp, col, val = (a.copy() for a in (g["row_ptr"], g["col"], g["val"]))
    if bad == "col_range":
        col[3] = 500
    elif bad == "row_ptr_order":
        rp[10], rp[11] = rp[11] + 1, rp[10]
    else:
        rp[-1] -= 1
    with pytest.raises(mp.MapiError) as ei:
        mp.mapi_pagerank(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(val).cuda(),
                         0.85, "mapi", max_iters=2)
    assert ei.value.status == 1


def test_full_size_2pow22_nodes_three_iterations():
    # the PageRank workload: n = 2^22, mean out-degree 16 (Zipf 2.1), uniform destinations
    n = 1 << 22
    print("[case] full pagerank generate", flush=True)
    g = synth.powerlaw_graph(n, seed=2022)
    rp, col, val = _dev(g)
    for method in ("mapi", "rpi"):
        print(f"[case] full pagerank {method}", flush=True)
        w, info = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=3)
        ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n), 3)
        wg = w.cpu().numpy()
        e, _ = report(f"pagerank {method} n=2^22 T=3", wg, ref.w)
        assert e <= TOL
        report(f"pagerank {method} n=2^22 T=3 deviation from 1/n", wg - 1 / n, ref.w - 1 / n)


@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_float64_iterate_matches_dense_oracle_and_the_deviation(method):
    # the FP64-iterate option: on 4096 nodes the iterate and its deviation from 1/n (the ranking
    # signal) match the dense brute-force FP64 oracle to summation order
    n, T = 4096, 12
    g = synth.powerlaw_graph(n, seed=9)
    rp, col, val = _dev(g)
    w, info = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=T, f64=True)
    assert w.dtype == torch.float64 and info["iters"] == T
    ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n), T, form="dense")
    wg = w.cpu().numpy()
    assert rel_l1(wg, ref.w) <= 1e-12
    assert rel_l1(wg - 1 / n, ref.w - 1 / n) <= 1e-9
    # a float64 start vector is used as given
    w0 = torch.from_numpy(np.full(n, 1.0 / n)).cuda()
    w2, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, w0=w0, max_iters=T, f64=True)
    np.testing.assert_array_equal(w2.cpu().numpy(), wg)


def test_float64_iterate_ranks_the_2pow22_graph():
    # n = 2^22, three MAPI iterations: the float64 iterate's top 100 is the oracle's (ties in the
    # oracle's scores at the cut would allow either order; the test checks there are none)
    n = 1 << 22
    print("[case] float64 pagerank generate", flush=True)
    g = synth.powerlaw_graph(n, seed=2022)
    rp, col, val = _dev(g)
    w, info = mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=3, f64=True)
    ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, "mapi", synth.uniform_start(n), 3)
    wg = w.cpu().numpy()
    assert rel_l1(wg - 1 / n, ref.w - 1 / n) <= 1e-9
    order = np.argsort(-ref.w, kind="stable")
    assert ref.w[order[99]] - ref.w[order[100]] > 1e-12 * ref.w[order[99]]
    assert set(np.argsort(-wg, kind="stable")[:100].tolist()) == set(order[:100].tolist())


def test_float64_iterate_rejects_float32_vectors():
    g = synth.powerlaw_graph(256, seed=3)
    rp, col, val = _dev(g)
    with pytest.raises(ValueError):
        mp.mapi_pagerank(rp, col, val, 0.85, "mapi", w0=torch.full((256,), 1 / 256, device="cuda"), f64=True)
