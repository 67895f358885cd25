"""mapi_solve_noalloc (every device buffer of the solve in the library's static scratch array)
through the C-ABI, against mapi_solve on the same context and against the FP64 oracle.

Calls follow one another with shrinking systems, so each call finds the previous call's
contents in the shared array: a solve that read a stale partial, state or iterate would
differ from mapi_solve's bits.  Tolerance against the oracle: relative l1 <= 1e-5 at the
same iteration count (the dense solve's bar)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from gpu_util import report, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5
ERR_ARG = 1

# (n, iterations, tol, stall): a fixed-iteration solve whose products form each iterate,
# a tolerance solve with the stall rule, a one-launch solve of a small system, and a
# smaller fixed solve again after it
CASES = [(5000, 25, 0.0, 0), (1500, 200, 1e-6, 8), (200, 60, 0.0, 0), (999, 12, 0.0, 0)]


def _case(n, seed):
    C64 = synth.dense_cov(n, 2 * n, seed=seed)
    return C64, synth.start_vector(n, seed + 1)


def test_noalloc_matches_mapi_solve_and_oracle_on_shrinking_calls():
    ctx = mp.Context()
    for k, (n, T, tol, stall) in enumerate(CASES):
        print(f"[case] noalloc n={n} T={T} tol={tol}", flush=True)
        A, w0 = _case(n, 100 + k)
        Ad, wd = to_dev(A), to_dev(w0)
        w1, i1 = mp.mapi_solve_noalloc(Ad, wd, max_iters=T, tol=tol, stall_iters=stall, ctx=ctx)
        w2, i2 = mp.mapi_solve(Ad, wd, max_iters=T, tol=tol, stall_iters=stall, ctx=ctx)
        assert i1 == i2
        np.testing.assert_array_equal(w1.cpu().numpy(), w2.cpu().numpy())
        ref = oracle.mapi(A.astype(np.float64), w0, i1["iters"])
        e, _ = report(f"noalloc n={n}", w1.cpu().numpy(), ref.w)
        assert e <= TOL


def test_noalloc_second_context_and_in_place_output():
    # another context on the same device uses the same array; w_out may alias w0
    ctx = mp.Context()
    A, w0 = _case(700, 7)
    Ad = to_dev(A)
    ref, _ = mp.mapi_solve(Ad, to_dev(w0), max_iters=15, ctx=ctx)
    wd = to_dev(w0)
    out, info = mp.mapi_solve_noalloc(Ad, wd, max_iters=15, w_out=wd, ctx=mp.Context())
    assert info["iters"] == 15 and out.data_ptr() == wd.data_ptr()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_rejects_systems_beyond_the_array():
    # the size check comes before any device work: the descriptor's pointer is never read
    ctx = mp.Context()
    n = 1 << 20
    assert ctx.workspace_size("solve", n) > 4 << 20
    dummy = torch.zeros(1024, dtype=torch.float32, device="cuda")
    d = mp.Dense(dummy.data_ptr(), n, n, n, mp.MAPI_F32, None)
    o = mp.Opts(5, 0.0, 0, 0, 0, 0)
    info = mp.Info()
    st = mp.lib().mapi_solve_noalloc(ctx.handle, C.byref(d), C.c_void_p(dummy.data_ptr()),
                                     C.c_void_p(dummy.data_ptr()), C.byref(o), C.byref(info))
    assert st == ERR_ARG
    assert b"static array" in mp.lib().mapi_last_error()
    # the largest order that fits still passes the check (no solve is run at that size here)
    fits = max(m for m in range(240000, 260000, 1000) if ctx.workspace_size("solve", m) <= 4 << 20)
    assert fits >= 240000
