"""GPU parity of the one-block solve of small float32 systems (n <= 256, Algorithm 1 and
eq. 1 run inside one launch) against the FP64 oracle and against the multi-kernel path of
the same solve (the size bucket pinned to a launch shape with mapi_tuning_set, which keeps
that path).  The two paths sum rows and norms in different orders, so iterates are compared
within the float32 tolerance; iteration counts, stop reasons and statuses must agree."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import cosine, rel_l1, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5
COS = 1 - 1e-6
SHAPE = dict(rows_per_wave=1, waves=4, blocks_per_cu=1, unroll=2, w_in_lds=1, nontemporal=0)


def _contexts(n):
    one, multi = mp.Context(), mp.Context()
    mp.mapi_tuning_set(mp.MAPI_F32, n, n, SHAPE, ctx=multi)
    return one, multi


def _solve(method, A, w0, ctx, **kw):
    if method == "rpi":
        return mp.rpi_solve(A, w0, ctx=ctx, **kw)
    return mp.mapi_solve(A, w0, op=method, ctx=ctx, **kw)


def _ref(method, A, w0, T, **kw):
    A = A.astype(np.float64)
    return oracle.rpi(A, w0, T, **kw) if method == "rpi" else oracle.mapi(A, w0, T, op=method, **kw)


@pytest.mark.parametrize("method", ["min1", "min2", "rpi"])
@pytest.mark.parametrize("n", [1, 3, 64, 100, 255, 256])
def test_fixed_iterations_match_oracle_and_multikernel(n, method):
    print(f"[case] small fixed {method} n={n}", flush=True)
    C = synth.dense_cov(n, 4 * n + 8, seed=100 + n)
    w0 = synth.start_vector(n, 200 + n)
    T = 40
    try:
        ref = _ref(method, C, w0, T)
    except oracle.OracleDegenerate:
        pytest.skip("normaliser zero for this draw (n = 1, min2)")
    one, multi = _contexts(n)
    Cd, wd = to_dev(C), to_dev(w0)
    w1, i1 = _solve(method, Cd, wd, one, max_iters=T)
    w2, i2 = _solve(method, Cd, wd, multi, max_iters=T)
    w1, w2 = w1.cpu().numpy(), w2.cpu().numpy()
    assert i1["iters"] == i2["iters"] == T and i1["status"] == i2["status"] == "OK"
    assert rel_l1(w1, ref.w) <= TOL and cosine(w1, ref.w) > COS
    assert rel_l1(w1, w2) <= TOL
    assert i1["norm"] == pytest.approx(i2["norm"], rel=1e-6)
    assert i1["norm"] == pytest.approx(ref.norms[-1], rel=1e-5)
    assert abs(i1["residual"] - ref.residuals[-1]) <= 1e-4 * ref.residuals[-1] + 1e-7


@pytest.mark.parametrize("method", ["min1", "rpi"])
def test_tolerance_and_stall_stops(method):
    A, _, _ = synth.planted_symmetric(200, [0.4], seed=31)
    w0 = synth.start_vector(200, 32)
    one, multi = _contexts(200)
    Ad, wd = to_dev(A), to_dev(w0)
    w1, i1 = _solve(method, Ad, wd, one, max_iters=500, tol=1e-6, check_every=5)
    w2, i2 = _solve(method, Ad, wd, multi, max_iters=500, tol=1e-6, check_every=5)
    assert i1["converged"] and i2["converged"] and i1["residual"] < 1e-6
    assert abs(i1["iters"] - i2["iters"]) <= 1
    ref = _ref(method, A, w0, i1["iters"])
    assert rel_l1(w1.cpu().numpy(), ref.w) <= TOL
    # a tolerance below the float32 floor: the stall rule ends both runs, unless the
    # iterate becomes exactly stationary first (residual 0, which is below any tolerance)
    s1, j1 = _solve(method, Ad, wd, one, max_iters=5000, tol=1e-30, stall_iters=20)
    s2, j2 = _solve(method, Ad, wd, multi, max_iters=5000, tol=1e-30, stall_iters=20)
    for j in (j1, j2):
        assert j["iters"] < 5000
        assert not j["converged"] or j["residual"] == 0.0
    assert rel_l1(s1.cpu().numpy(), s2.cpu().numpy()) <= 1e-4


def test_final_l2_zero_iterations_in_place_and_degenerate():
    n = 128
    C = synth.dense_cov(n, 600, seed=41)
    w0 = synth.start_vector(n, 42)
    one, multi = _contexts(n)
    Cd = to_dev(C)
    w1, _ = mp.mapi_solve(Cd, to_dev(w0), max_iters=25, final_l2=True, ctx=one)
    w2, _ = mp.mapi_solve(Cd, to_dev(w0), max_iters=25, final_l2=True, ctx=multi)
    ref = oracle.mapi(C.astype(np.float64), w0, 25, final_l2=True)
    assert rel_l1(w1.cpu().numpy(), ref.w) <= TOL and rel_l1(w1.cpu().numpy(), w2.cpu().numpy()) <= TOL
    assert float(torch.linalg.norm(w1.double())) == pytest.approx(1.0, abs=1e-6)
    # no iterations: the start vector comes back
    w, info = mp.mapi_solve(Cd, to_dev(w0), max_iters=0, ctx=one)
    assert info["iters"] == 0
    np.testing.assert_array_equal(w.cpu().numpy(), w0)
    # the output may be the start vector's own buffer
    wd = to_dev(w0)
    w3, _ = mp.mapi_solve(Cd, wd, max_iters=25, w_out=wd, ctx=one)
    w4, _ = mp.mapi_solve(Cd, to_dev(w0), max_iters=25, ctx=one)
    np.testing.assert_array_equal(w3.cpu().numpy(), w4.cpu().numpy())
    # a zero matrix: the first normaliser is zero on both paths
    Z = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    for ctx in (one, multi):
        with pytest.raises(mp.MapiError) as ei:
            mp.mapi_solve(Z, to_dev(w0), max_iters=10, ctx=ctx)
        assert ei.value.status == 4


def test_repeat_is_bitwise_deterministic():
    C = synth.dense_cov(256, 1024, seed=11)
    w0 = synth.start_vector(256, 12)
    one, _ = _contexts(256)
    a, ia = mp.mapi_solve(to_dev(C), to_dev(w0), max_iters=200, ctx=one)
    b, ib = mp.mapi_solve(to_dev(C), to_dev(w0), max_iters=200, ctx=one)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert ia == ib


def test_long_solves_launch_per_iteration():
    # more than 65536 allowed iterations: the solve launches a product per iteration, so no
    # single kernel runs for long; a tolerance ends it early
    A, _, _ = synth.planted_symmetric(64, [0.4], seed=51)
    w0 = synth.start_vector(64, 52)
    ctx = mp.Context()
    ctx.timing(True)
    ctx.timing_reset()
    w, info = mp.mapi_solve(to_dev(A), to_dev(w0), max_iters=100000, tol=1e-6, ctx=ctx)
    _, launches = ctx.timing_get("mavp")
    ctx.timing(False)
    assert info["converged"] and launches >= info["iters"] > 1
    ref = oracle.mapi(A.astype(np.float64), w0, info["iters"])
    assert rel_l1(w.cpu().numpy(), ref.w) <= TOL


def test_small_solve_min1_xor_form_same_bits(monkeypatch):
    # the one-block solve's min1 term as sign flip, med3 and add (MAPI_MIN1_FORM=xor) gives the
    # bits of the FMA-by-+-1 form
    import synth
    for n in (64, 200, 256):
        C = to_dev(synth.dense_cov(n, 3 * n, seed=n))
        w0 = to_dev(synth.start_vector(n, n + 1))
        a, ia = mp.mapi_solve(C, w0, max_iters=40, tol=1e-7)
        monkeypatch.setenv("MAPI_MIN1_FORM", "xor")
        b, ib = mp.mapi_solve(C, w0, max_iters=40, tol=1e-7)
        monkeypatch.delenv("MAPI_MIN1_FORM")
        assert ia["iters"] == ib["iters"]
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
