"""Caller-owned device workspace (mapi_workspace_size / mapi_set_workspace) through the C-ABI.

Each call kind runs twice on the same inputs: once in a context that allocates its own
device memory, once in a context given a torch tensor of exactly the size
mapi_workspace_size reports (pre-filled with NaN bytes, so that a buffer read before it
is written shows up).  The results must be bitwise identical, the workspace must have
been written, and a region 256 bytes too small must fail with MAPI_ERR_ARG before any
device work.  The oracle parity of each call is covered by its own test module.
"""
import numpy as np
import pytest

import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

ERR_ARG = 1


def _workspace(nbytes):
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    buf.fill_(0xFF)                 # every float and double read from it is NaN
    return buf


def _pair(kind, n, nnz=0, extra=0):
    """An own-memory context, a context on an exactly sized workspace, and that workspace."""
    own = mp.Context()
    user = mp.Context()
    nbytes = user.workspace_size(kind, n, nnz) + extra
    ws = _workspace(nbytes)
    user.set_workspace(ws)
    return own, user, ws


def _written(ws):
    return bool((ws != 0xFF).any().item())


def _too_small(kind, n, nnz, call, extra=0):
    ctx = mp.Context()
    nbytes = ctx.workspace_size(kind, n, nnz) + extra
    ws = _workspace(nbytes - 256)
    ctx.set_workspace(ws)
    with pytest.raises(mp.MapiError) as e:
        call(ctx)
    assert e.value.status == ERR_ARG and "workspace" in str(e.value)
    assert not _written(ws)


@pytest.mark.parametrize("n,method,tol", [(200, "mapi", 0.0), (1003, "mapi", 0.0), (1003, "mapi", 1e-6),
                                          (777, "rpi", 0.0)])
def test_solve_in_caller_workspace(n, method, tol):
    print(f"[case] workspace solve n={n} {method} tol={tol}", flush=True)
    A = to_dev(synth.dense_cov(n, 2 * n, seed=n))
    w0 = to_dev(synth.start_vector(n, n + 1))
    fn = mp.mapi_solve if method == "mapi" else mp.rpi_solve
    own, user, ws = _pair("solve", n)
    a, ia = fn(A, w0, max_iters=40, tol=tol, ctx=own)
    b, ib = fn(A, w0, max_iters=40, tol=tol, ctx=user)
    assert ia == ib and _written(ws)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    _too_small("solve", n, 0, lambda c: fn(A, w0, max_iters=5, ctx=c))


def test_hybrid_in_caller_workspace():
    n = 600
    A = to_dev(synth.dense_cov(n, 1500, seed=5))
    w0 = to_dev(synth.start_vector(n, 6))
    own, user, ws = _pair("hybrid", n)
    a = mp.mapi_hybrid_solve(A, w0, mapi_iters=10, rpi_iters=15, ctx=own)
    b = mp.mapi_hybrid_solve(A, w0, mapi_iters=10, rpi_iters=15, ctx=user)
    assert a[1:] == b[1:] and _written(ws)
    np.testing.assert_array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    _too_small("hybrid", n, 0, lambda c: mp.mapi_hybrid_solve(A, w0, mapi_iters=2, rpi_iters=2, ctx=c))


@pytest.mark.parametrize("f64", [False, True])
@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_pagerank_in_caller_workspace(method, f64):
    g = synth.powerlaw_graph(3000, seed=21)
    rp, col, val = (torch.from_numpy(g[k]).cuda() for k in ("row_ptr", "col", "val"))
    kind = "pagerank_f64" if f64 else "pagerank"
    own, user, ws = _pair(kind, g["n"], g["col"].size)
    a, ia = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=12, f64=f64, ctx=own)
    b, ib = mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=12, f64=f64, ctx=user)
    assert ia == ib and _written(ws)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    _too_small(kind, g["n"], g["col"].size, lambda c: mp.mapi_pagerank(rp, col, val, 0.85, method, max_iters=2, f64=f64, ctx=c))


@pytest.mark.parametrize("op", ["min1", "dot"])
def test_mingram_in_caller_workspace(op):
    # 4099 samples split into several chunks whose float64 partial tiles are workspace
    D, N = 200, 4099
    X = to_dev(synth.pca_data(D, N, seed=4))
    own, user, ws = _pair("mingram", D, N)
    a = mp.mapi_mingram(X, 1.0 / N, op, ctx=own)
    b = mp.mapi_mingram(X, 1.0 / N, op, ctx=user)
    assert _written(ws)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    if op == "min1":   # the size covers the larger (min-form) split; the dot build needs less
        _too_small("mingram", D, N, lambda c: mp.mapi_mingram(X, 1.0 / N, op, ctx=c))


@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_pca_in_caller_workspace(method):
    D, N, k = 256, 3000, 3
    X = to_dev(synth.pca_data(D, N, seed=8))
    W0 = torch.from_numpy(synth.start_vectors(D, k, seed=9)).cuda()
    own = mp.Context()
    user = mp.Context()
    nbytes = user.workspace_size("pca", D, N) + (k - 1) * user.workspace_size("pca_vector", D)
    ws = _workspace(nbytes)
    user.set_workspace(ws)
    a, ia = mp.mapi_pca_topk(X, k, W0, method, max_iters=25, ctx=own)
    b, ib = mp.mapi_pca_topk(X, k, W0, method, max_iters=25, ctx=user)
    assert ia == ib and _written(ws)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    if method == "mapi":   # the size covers the min-form build's partial tiles; RPI's need less
        extra = (k - 1) * user.workspace_size("pca_vector", D)
        _too_small("pca", D, N, lambda c: mp.mapi_pca_topk(X, k, W0, method, max_iters=2, ctx=c), extra=extra)


@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_image_in_caller_workspace(method):
    D, N = 24, 10
    _, V = synth.occluded_images(D, N, seed=3)
    Vd = torch.from_numpy(V).cuda()
    w0 = to_dev(synth.start_vector(D * D, 4))
    own, user, ws = _pair("image", D * D, N)
    Ra, Wa, ia = mp.mapi_image_reconstruct(Vd, w0, method, max_iters=20, ctx=own)
    Rb, Wb, ib = mp.mapi_image_reconstruct(Vd, w0, method, max_iters=20, ctx=user)
    assert ia == ib and _written(ws)
    np.testing.assert_array_equal(Ra.cpu().numpy(), Rb.cpu().numpy())
    np.testing.assert_array_equal(Wa.cpu().numpy(), Wb.cpu().numpy())
    if method == "mapi":
        _too_small("image", D * D, N, lambda c: mp.mapi_image_reconstruct(Vd, w0, method, max_iters=2, ctx=c))


@pytest.mark.parametrize("kind", ["minibatch", "minibatch_min"])
def test_minibatch_in_caller_workspace(kind):
    # with the least workspace the batch matrices of one step of t are built per launch;
    # the recurrence is the same, so the bits are too
    rng = np.random.default_rng(17)
    N, D, runs, T, s = 400, 12, 3, 9, 20
    X = to_dev(rng.standard_normal((N, D)).astype(np.float32))
    batches = torch.from_numpy(synth.minibatch_indices(runs, T, s, N, seed=2)).cuda()
    W0 = torch.from_numpy(np.stack([synth.start_vector(D, 30 + r) for r in range(runs)])).cuda()
    own, user, ws = _pair(kind, D, runs)
    a, ia = mp.mapi_minibatch(X, batches, 0.2, W0, ctx=own)
    b, ib = mp.mapi_minibatch(X, batches, 0.2, W0, ctx=user)
    assert ia == ib and _written(ws)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    if kind == "minibatch_min":
        _too_small(kind, D, runs, lambda c: mp.mapi_minibatch(X, batches, 0.2, W0, ctx=c))


@pytest.mark.parametrize("op", ["min1", "min2"])
def test_factored_in_caller_workspace(op):
    D, N = 150, 2050
    X = to_dev(synth.pca_data(D, N, seed=14))
    w0 = to_dev(synth.start_vector(D, 15))
    own, user, ws = _pair("factored", D, N)
    a, ia = mp.mapi_factored_solve(X, w0, max_iters=9, op=op, ctx=own)
    b, ib = mp.mapi_factored_solve(X, w0, max_iters=9, op=op, ctx=user)
    assert ia == ib and _written(ws)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    _too_small("factored", D, N, lambda c: mp.mapi_factored_solve(X, w0, max_iters=2, op=op, ctx=c))


def test_product_calls_in_caller_workspace():
    n = 1000
    A = to_dev(synth.dense_cov(n, 1200, seed=12))
    wbuf = torch.from_numpy(synth.start_vector(n + 1, 13)).cuda()
    w = wbuf[1:]                    # 4-byte aligned only: mapi_mavp copies it into workspace
    own, user, ws = _pair("product", n, n)
    a = mp.mapi_mavp(A, w, ctx=own)
    b = mp.mapi_mavp(A, w, ctx=user)
    assert _written(ws)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    shape, _ = mp.mapi_autotune_dense(A, reps=1, ctx=user)
    assert shape["waves"] in (4, 8)
    assert mp.mapi_read_reference(A, reps=1, ctx=user) > 0
    _too_small("product", n, n, lambda c: mp.mapi_autotune_dense(A, reps=1, ctx=c))


def test_batched_in_caller_workspace():
    g = synth.powerlaw_graph(2000, seed=31)
    rp, col, val = (torch.from_numpy(g[k]).cuda() for k in ("row_ptr", "col", "val"))

    def problems():
        return [mp.problem_generated(700, 3, "f32", "mapi", max_iters=30),
                mp.problem_generated(300, 4, "bf16", "rpi", max_iters=30),
                mp.problem_csr(rp, col, val, 0.85, "mapi", max_iters=10)]

    own = mp.Context()
    user = mp.Context()
    pa, pb = problems(), problems()
    nbytes = mp.mapi_solve_batched_workspace_size(pb, ctx=user)
    ws = _workspace(nbytes)
    user.set_workspace(ws)
    ia = mp.mapi_solve_batched(pa, ctx=own)
    ib = mp.mapi_solve_batched(pb, ctx=user)
    assert ia == ib and _written(ws)
    for p, q in zip(pa, pb):
        np.testing.assert_array_equal(p.out.cpu().numpy(), q.out.cpu().numpy())
    small = mp.Context()
    tiny = _workspace(nbytes - 256)
    small.set_workspace(tiny)
    with pytest.raises(mp.MapiError) as e:
        mp.mapi_solve_batched(problems(), ctx=small)
    assert e.value.status == ERR_ARG
    assert not _written(tiny)


def test_workspace_release_and_bad_arguments():
    ctx = mp.Context()
    n = 500
    A = to_dev(synth.dense_cov(n, 900, seed=40))
    w0 = to_dev(synth.start_vector(n, 41))
    a, _ = mp.mapi_solve(A, w0, max_iters=10, ctx=ctx)
    ws = _workspace(ctx.workspace_size("solve", n))
    ctx.set_workspace(ws)
    b, _ = mp.mapi_solve(A, w0, max_iters=10, ctx=ctx)
    ctx.set_workspace(None)          # back to context-owned memory
    c, _ = mp.mapi_solve(A, w0, max_iters=10, ctx=ctx)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    np.testing.assert_array_equal(a.cpu().numpy(), c.cpu().numpy())
    L = mp.lib()
    import ctypes as C
    assert L.mapi_set_workspace(ctx.handle, C.c_void_p(ws.data_ptr() + 16), 4096) == ERR_ARG   # misaligned
    assert L.mapi_set_workspace(ctx.handle, C.c_void_p(ws.data_ptr()), 0) == ERR_ARG           # empty
    out = C.c_size_t()
    assert L.mapi_workspace_size(ctx.handle, 99, 10, 0, C.byref(out)) == ERR_ARG             # unknown kind
    assert L.mapi_workspace_size(ctx.handle, 0, 0, 0, C.byref(out)) == ERR_ARG               # n = 0
    # the bound covers every launch shape: a larger system never needs less
    sizes = [ctx.workspace_size("solve", m) for m in (1, 255, 256, 4096, 16384, 1 << 20)]
    assert sizes == sorted(sizes)
