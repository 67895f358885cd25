"""GPU tests of the continuous-batching server: results equal the same problem solved alone,
admission under a memory budget, rejection of oversize requests, and statistics."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel_l1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5


def _alone(prob_factory):
    """Solve one problem by itself with a fresh context (default tile heights)."""
    ctx = mp.Context()
    p = prob_factory()
    info = mp.mapi_solve_batched([p], ctx=ctx)[0]
    out = p.out.cpu().numpy().copy()
    ctx.close()
    return out, info


def test_serve_results_equal_alone_and_oracle():
    graphs = {n: synth.powerlaw_graph(n, seed=n) for n in (1500, 30000)}
    specs = []
    rng = np.random.default_rng(3)
    for i in range(36):
        if i % 4 == 3:
            n = 1500 if i % 8 == 3 else 30000
            specs.append(("csr", n, ["mapi", "rpi"][i % 2], 0))
        else:
            n = int(np.exp(rng.uniform(np.log(64), np.log(3000))))
            specs.append(("gen", n, ["mapi", "rpi"][(i // 2) % 2], ["f32", "bf16"][i % 2]))
    srv = mp.Server(budget_bytes=4 << 30)
    tickets, outs = [], []
    for i, (kind, n, meth, dt) in enumerate(specs):
        if kind == "csr":
            g = graphs[n]
            prob = mp.request_csr_host(g["row_ptr"], g["col"], g["val"], 0.85, meth, max_iters=200, tol=1e-7)
        else:
            prob = mp.request_generated(n, 900 + i, dt, meth, max_iters=300, tol=1e-6)
        out = np.zeros(n, np.float32)
        tickets.append(srv.submit(prob, out))
        outs.append(out)
        time.sleep(0.002 * (i % 3))                     # staggered arrivals join the running kernel
    results = [srv.wait(t, timeout_us=60_000_000) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(specs) and stats["rejected"] == 0
    print(f"[serve] {stats}", flush=True)
    for i, ((kind, n, meth, dt), res, out) in enumerate(zip(specs, results, outs)):
        assert res is not None and res["status"] == "OK", (i, res)
        if kind == "csr":
            g = graphs[n]
            rp, col, val = (torch.from_numpy(g[x]).cuda() for x in ("row_ptr", "col", "val"))
            w_alone, info = _alone(lambda: mp.problem_csr(rp, col, val, 0.85, meth, max_iters=200, tol=1e-7))
        else:
            w_alone, info = _alone(lambda: mp.problem_generated(n, 900 + i, dt, meth, max_iters=300, tol=1e-6))
        assert info["iters"] == res["iters"], (i, info, res)
        np.testing.assert_array_equal(out, w_alone)
        if kind == "gen" and n <= 1500 and i % 5 == 0:
            A, w0 = synth.generated_dense(n, 900 + i)
            if dt == "bf16":
                A = oracle.bf16_decode(oracle.bf16_encode(A))
            fn = oracle.mapi if meth == "mapi" else oracle.rpi
            ref = fn(A.astype(np.float64), w0, res["iters"])
            assert rel_l1(out, ref.w) <= TOL


def test_serve_rejects_request_larger_than_budget():
    srv = mp.Server(budget_bytes=64 << 20)
    with pytest.raises(mp.MapiError) as ei:
        srv.submit(mp.request_generated(8192, 1, "f32"), np.zeros(8192, np.float32))
    assert ei.value.status == 5
    srv.close()


def test_serve_admission_respects_small_budget():
    # each n = 2048 float32 request needs about 16.1 MiB; the budget admits two at a time
    srv = mp.Server(budget_bytes=40 << 20)
    outs, ts = [], []
    for i in range(10):
        out = np.zeros(2048, np.float32)
        ts.append(srv.submit(mp.request_generated(2048, 40 + i, "f32", "rpi", max_iters=100, tol=1e-6), out))
        outs.append(out)
    res = [srv.wait(t, timeout_us=60_000_000) for t in ts]
    st = srv.stats()
    srv.close()
    assert all(r["status"] == "OK" for r in res)
    assert st["peak_bytes"] <= 40 << 20 and st["completed"] == 10
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_serve_invalid_request_fails_alone():
    g = synth.powerlaw_graph(800, seed=2)
    bad_col = g["col"].copy()
    bad_col[5] = 10_000
    srv = mp.Server(budget_bytes=1 << 30)
    out_bad = np.zeros(800, np.float32)
    out_ok = np.zeros(900, np.float32)
    t_bad = srv.submit(mp.request_csr_host(g["row_ptr"], bad_col, g["val"], 0.85, "mapi"), out_bad)
    t_ok = srv.submit(mp.request_generated(900, 5, "f32", "mapi", max_iters=50, tol=0.0), out_ok)
    r_bad = srv.wait(t_bad, timeout_us=30_000_000)
    r_ok = srv.wait(t_ok, timeout_us=30_000_000)
    srv.close()
    assert r_bad["status"] == "ERR_ARG"
    assert r_ok["status"] == "OK" and r_ok["iters"] == 50


def test_serve_rejects_pageable_csr_arrays():
    # the kernel reads a served request's CSR arrays from pinned host memory itself
    import ctypes as C
    g = synth.powerlaw_graph(300, seed=4)
    prob = mp.request_csr_host(g["row_ptr"], g["col"], g["val"], 0.85, "mapi")
    rp, col, val = (np.ascontiguousarray(g[k]) for k in ("row_ptr", "col", "val"))
    prob.H = mp.Csr(300, col.size, rp.ctypes.data, col.ctypes.data, val.ctypes.data)   # pageable numpy memory
    srv = mp.Server(budget_bytes=256 << 20)
    out = np.zeros(300, np.float32)
    req = mp.Request(prob, out.ctypes.data)
    t = C.c_uint64()
    st = mp.lib().mapi_serve_submit(srv.handle, C.byref(req), C.byref(t))
    srv.close()
    assert mp.STATUS.get(st, st) == "ERR_ARG"


def test_serve_pagerank_checks_on_device():
    # row_ptr not ending at nnz, a decreasing row_ptr and an out-of-range column are each
    # found by the kernel's admission phases; valid requests in the same mix are unaffected
    g = synth.powerlaw_graph(20000, seed=6)
    bad = []
    rp = g["row_ptr"].copy(); rp[-1] -= 1
    bad.append((rp, g["col"], g["val"]))
    rp = g["row_ptr"].copy(); rp[100], rp[101] = rp[101], rp[100] - 1
    bad.append((rp, g["col"], g["val"]))
    col = g["col"].copy(); col[-1] = -3
    bad.append((g["row_ptr"], col, g["val"]))
    srv = mp.Server(budget_bytes=1 << 30)
    tickets = []
    for i in range(6):
        if i % 2:
            r, c, v = bad[i // 2]
            tickets.append(("bad", srv.submit(mp.request_csr_host(r, c, v, 0.85, "rpi"), np.zeros(20000, np.float32))))
        else:
            out = np.zeros(20000, np.float32)
            tickets.append(("ok", srv.submit(mp.request_csr_host(g["row_ptr"], g["col"], g["val"], 0.85, "rpi",
                                                                  max_iters=60, tol=1e-7), out), out))
    res = [(x[0], srv.wait(x[1], timeout_us=60_000_000)) + tuple(x[2:]) for x in tickets]
    srv.close()
    rp_d, col_d, val_d = (torch.from_numpy(g[x]).cuda() for x in ("row_ptr", "col", "val"))
    w_alone, info = _alone(lambda: mp.problem_csr(rp_d, col_d, val_d, 0.85, "rpi", max_iters=60, tol=1e-7))
    for r in res:
        if r[0] == "bad":
            assert r[1]["status"] == "ERR_ARG"
        else:
            assert r[1]["status"] == "OK" and r[1]["iters"] == info["iters"]
            np.testing.assert_array_equal(r[2], w_alone)
