"""GPU parity of the column-split PageRank product (eq. 11 split sums, 8 source blocks, per-block
row sums added in block order) against the FP64 oracle, and its agreement with the plain CSR
product.  Small graphs are forced onto the split layout (mapi_pagerank_split_config(1)); the
2^22-node graph takes it by default."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel_l1, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5


def _dev(g):
    return (torch.from_numpy(np.ascontiguousarray(g["row_ptr"])).cuda(),
            torch.from_numpy(np.ascontiguousarray(g["col"])).cuda(),
            torch.from_numpy(np.ascontiguousarray(g["val"])).cuda())


def _ctx(split, after=0):
    # split: every graph takes the split layout, built before the first product (after = 0)
    # unless `after` says otherwise
    c = mp.Context()
    mp.mapi_pagerank_split_config(1 if split else 0, ctx=c)
    mp.mapi_pagerank_split_after(after, ctx=c)
    return c


@pytest.mark.parametrize("f64", [False, True])
@pytest.mark.parametrize("method", ["mapi", "rpi"])
@pytest.mark.parametrize("n,T", [(4096, 1), (4096, 12), (4099, 7), (61, 5)])
def test_split_matches_dense_oracle(n, T, method, f64):
    # 4099 and 61 nodes: blocks of 513 and 8 sources, a ragged last block and a partial
    # last chunk of 64 rows
    print(f"[case] split pagerank n={n} T={T} {method} f64={f64}", flush=True)
    g = synth.powerlaw_graph(n, seed=n + 5)
    rp, col, val = _dev(g)
    w, info = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=T, f64=f64, ctx=_ctx(True))
    assert info["iters"] == T
    ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n), T,
                          form="dense")
    wg = w.cpu().numpy()
    e, _ = report(f"split pagerank {method} n={n} T={T} f64={f64}", wg, ref.w)
    assert e <= (1e-12 if f64 else TOL)
    if f64:
        assert rel_l1(wg - 1 / n, ref.w - 1 / n) <= 1e-9
    # the plain product on the same graph: the same iterate up to the order of the row sums
    w2, info2 = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=T, f64=f64, ctx=_ctx(False))
    assert info2["iters"] == T
    assert rel_l1(wg, w2.cpu().numpy()) <= (1e-13 if f64 else 1e-6)


def test_split_with_unsorted_rows_tolerance_stop_and_dangling():
    # columns within a row in reverse order (the input contract allows any order), a
    # tolerance stop, and the graph's 5 % dangling nodes
    n = 5000
    g = synth.powerlaw_graph(n, seed=77)
    col = g["col"].copy()
    val = g["val"].copy()
    for i in range(n):
        a, b = g["row_ptr"][i], g["row_ptr"][i + 1]
        col[a:b] = col[a:b][::-1]
        val[a:b] = val[a:b][::-1]
    h = dict(row_ptr=g["row_ptr"], col=col, val=val)
    rp, cd, vd = _dev(h)
    for method in ("mapi", "rpi"):
        w, info = mp.mapi_pagerank(rp, cd, vd, 0.85, method, max_iters=200, tol=1e-7, check_every=4,
                                   ctx=_ctx(True))
        assert info["converged"]
        ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n),
                              info["iters"])
        e, _ = report(f"split pagerank unsorted {method}", w.cpu().numpy(), ref.w)
        assert e <= TOL


def test_long_block_row_keeps_the_plain_product():
    # row 0 holds 300 links from block 0's sources (at n = 4096 a block has 512 sources):
    # too long for the split layout's byte lengths, so the plain product runs -- same bits
    n = 4096
    edges = [(j, 0) for j in range(1, 301)] + [(j, (j * 7) % n) for j in range(n) if (j * 7) % n != j]
    g = synth.tiny_graph(edges, n)
    rp, col, val = _dev(g)
    for method in ("mapi", "rpi"):
        a, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=6, ctx=_ctx(True))
        b, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=6, ctx=_ctx(False))
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n), 6,
                              form="dense")
        assert rel_l1(a.cpu().numpy(), ref.w) <= TOL


def test_chunk_larger_than_the_lds_assembly_buffer():
    # rows 0..63 (one chunk of 64 rows) hold 30 links from each of the 8 source blocks:
    # 15360 links in one chunk, more than the layout scatter assembles in LDS (1536), so
    # its entries are written one by one, while every block row (30 links) stays short
    # enough for the split layout; the other chunks take the LDS assembly
    n = 4096
    edges = [(k * 512 + (i * 13 + t * 17) % 512, i) for i in range(64) for k in range(8) for t in range(30)]
    edges += [(j, (j * 7) % n) for j in range(n)]
    g = synth.tiny_graph([(j, i) for j, i in edges if j != i], n)
    assert int(g["row_ptr"][64]) > 1536
    rp, col, val = _dev(g)
    for f64 in (False, True):
        for method in ("mapi", "rpi"):
            a, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=6, f64=f64, ctx=_ctx(True))
            b, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=6, f64=f64, ctx=_ctx(False))
            ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n), 6,
                                  form="dense")
            e, _ = report(f"pagerank split big chunk {method} f64={f64}", a.cpu().numpy(), ref.w)
            assert e <= (1e-12 if f64 else TOL)
            assert rel_l1(a.cpu().numpy(), b.cpu().numpy()) <= (1e-13 if f64 else 1e-6)


def test_split_repeat_is_bitwise_deterministic():
    n = 20000
    g = synth.powerlaw_graph(n, seed=3)
    rp, col, val = _dev(g)
    c = _ctx(True)
    a, _ = mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=9, ctx=c)
    b, _ = mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=9, ctx=c)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_full_size_split_against_csr_oracle_and_plain_product():
    # the PageRank workload at n = 2^22 takes the split layout by default: three MAPI and RPI
    # iterations against the CSR oracle, and against the plain product
    n = 1 << 22
    print("[case] split pagerank 2^22 generate", flush=True)
    g = synth.powerlaw_graph(n, seed=2022)
    rp, col, val = _dev(g)
    c_split, c_plain = mp.Context(), _ctx(False)
    mp.mapi_pagerank_split_after(0, ctx=c_split)     # the default layout rule, split from the first product
    for method in ("mapi", "rpi"):
        print(f"[case] split pagerank 2^22 {method}", flush=True)
        w, info = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=3, ctx=c_split)
        ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n), 3)
        wg = w.cpu().numpy()
        e, _ = report(f"split pagerank {method} n=2^22 T=3", wg, ref.w)
        assert e <= TOL
        w2, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=3, ctx=c_plain)
        assert rel_l1(wg, w2.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_split_built_after_the_first_products(method):
    # the default policy: plain products for the first `after` iterations, then the split layout
    # if the solve is still running.  T <= after: the plain product's bits; T > after: against
    # the oracle, close to both single-layout runs, and bitwise repeatable
    n = 5000
    g = synth.powerlaw_graph(n, seed=31)
    rp, col, val = _dev(g)
    lazy = _ctx(True, after=4)
    a, ia = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=4, ctx=lazy)
    b, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=4, ctx=_ctx(False))
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    T = 11
    w, info = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=T, ctx=lazy)
    assert info["iters"] == T
    ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, method, synth.uniform_start(n), T,
                          form="dense")
    e, _ = report(f"lazy split pagerank {method} T={T}", w.cpu().numpy(), ref.w)
    assert e <= TOL
    for other in (_ctx(True), _ctx(False)):
        w2, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=T, ctx=other)
        assert rel_l1(w.cpu().numpy(), w2.cpu().numpy()) <= 1e-6
    w3, _ = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=T, ctx=lazy)
    np.testing.assert_array_equal(w.cpu().numpy(), w3.cpu().numpy())
    # a tolerance solve that stops before the switch: the plain product's bits and count
    t1, i1 = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=300, tol=1e-2, check_every=1, ctx=_ctx(True, 50))
    t2, i2 = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=300, tol=1e-2, check_every=1, ctx=_ctx(False))
    assert i1["iters"] == i2["iters"] < 50
    np.testing.assert_array_equal(t1.cpu().numpy(), t2.cpu().numpy())


def test_split_after_rejects_negative():
    with pytest.raises(mp.MapiError) as ei:
        mp.mapi_pagerank_split_after(-1)
    assert ei.value.status == 1
