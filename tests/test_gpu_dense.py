"""GPU parity of the dense path (product, MAPI, RPI, storage formats) against the FP64 oracle.

Calls go through the C-ABI (libmapi.so via the ctypes binding).  Tolerances:
bit-exact where every partial sum is exact in float32 (dyadic inputs) and for
the storage encoders; otherwise relative l1 <= 1e-5 and cosine > 1 - 1e-6
against the oracle iterate at the same iteration count.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import cosine, rel_l1, report, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5
COS = 1 - 1e-6


def _stored(A32, dtype):
    """Device copy of A in storage `dtype` plus the float32 matrix it decodes to (oracle side)."""
    if dtype == "f32":
        return to_dev(A32), None, A32
    if dtype == "bf16":
        q = oracle.bf16_encode(A32)
        return to_dev(q.view(np.int16)), None, oracle.bf16_decode(q)
    q = oracle.e4m3fn_encode(A32)
    s = np.ones(A32.shape[0], np.float32)
    return to_dev(q), to_dev(s), oracle.fp8_rows_dequantize(q, s)


SHAPES = [(1, 1), (3, 5), (64, 100), (257, 1031), (1000, 4099), (4096, 256), (33, 16400)]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("op", ["min1", "min2", "diamond", "dot"])
@pytest.mark.parametrize("shape", SHAPES)
def test_mavp_dyadic_bitexact(dtype, op, shape):
    m, n = shape
    print(f"[case] mavp dyadic {dtype} {op} {shape}", flush=True)
    A = synth.dyadic_matrix(m, n, seed=m * 7 + n)
    w = synth.dyadic_vector(n, seed=m + 3 * n + 1)
    Ad, rs, Aref = _stored(A, dtype)
    np.testing.assert_array_equal(Aref, A)          # dyadic values are exact in every format
    y = mp.mapi_mavp(Ad, to_dev(w), op=op, row_scale=rs).cpu().numpy()
    ref = oracle.mavp(A, w, op).astype(np.float32)
    np.testing.assert_array_equal(y, ref)


def test_fp8_decode_every_code():
    codes = np.arange(256, dtype=np.uint8)
    codes[[0x7F, 0xFF]] = 0
    A = np.zeros((256, 16), np.uint8)
    A[:, 0] = codes
    w = np.full(16, 1e30, np.float32)               # min1(a, w) = a for every finite a
    for scale in (1.0, 3.0):
        s = np.full(256, scale, np.float32)
        y = mp.mapi_mavp(to_dev(A), to_dev(w), "min1", row_scale=to_dev(s)).cpu().numpy()
        ref = (np.float32(scale) * oracle.e4m3fn_decode(codes)).astype(np.float32)
        np.testing.assert_array_equal(y, ref)


def test_quantizers_bitexact():
    rng = np.random.default_rng(5)
    A = (rng.standard_normal((300, 1001)) * np.exp(rng.uniform(-8, 8, (300, 1)))).astype(np.float32)
    A[7] = 0.0
    A[8, :5] = [448.0 * 3, -1e-30, 0.0, -0.0, 1e-8]
    Ad = to_dev(A)
    qb, _ = mp.mapi_quantize(Ad, "bf16")
    np.testing.assert_array_equal(qb.cpu().numpy().view(np.uint16), oracle.bf16_encode(A))
    q8, s8 = mp.mapi_quantize(Ad, "fp8")
    q_ref, s_ref = oracle.fp8_rows_quantize(A)
    np.testing.assert_array_equal(s8.cpu().numpy(), s_ref)
    np.testing.assert_array_equal(q8.cpu().numpy(), q_ref)


@pytest.mark.parametrize("T", [1, 3, 20, 200])
def test_mapi_and_rpi_match_oracle_n256(T):
    # the n = 256 workload: C = X X^T / 1024, rows of X centred, b0 ~ U(-1, 1) scaled to unit l2
    C = synth.dense_cov(256, 1024, seed=11)
    w0 = synth.start_vector(256, 12)
    Cd, wd = to_dev(C), to_dev(w0)
    w, info = mp.mapi_solve(Cd, wd, max_iters=T)
    assert info["iters"] == T and info["status"] == "OK"
    ref = oracle.mapi(C.astype(np.float64), w0, T)
    e, c = report(f"mapi n=256 T={T}", w.cpu().numpy(), ref.w)
    assert e <= TOL and c > COS
    assert abs(info["residual"] - ref.residuals[-1]) <= 1e-4 * ref.residuals[-1] + 1e-7
    b, info_r = mp.rpi_solve(Cd, wd, max_iters=T)
    ref_r = oracle.rpi(C.astype(np.float64), w0, T)
    e, c = report(f"rpi n=256 T={T}", b.cpu().numpy(), ref_r.w)
    assert e <= TOL and c > COS
    assert info_r["norm"] == pytest.approx(ref_r.norms[-1], rel=1e-6)


def test_tolerance_stop_compared_at_gpu_iteration_count():
    A, Q, d = synth.planted_symmetric(300, [0.4], seed=21)
    w0 = synth.start_vector(300, 22)
    for solver, ref_fn in ((mp.mapi_solve, oracle.mapi), (mp.rpi_solve, oracle.rpi)):
        w, info = solver(to_dev(A), to_dev(w0), max_iters=500, tol=1e-6, check_every=7)
        assert info["converged"] and info["residual"] < 1e-6
        t = info["iters"]
        ref = ref_fn(A.astype(np.float64), w0, t)
        assert rel_l1(w.cpu().numpy(), ref.w) <= TOL
        stop = ref_fn(A.astype(np.float64), w0, 500, tol=1e-6)
        assert abs(stop.iters - t) <= 2


@pytest.mark.parametrize("n", [1, 2, 7, 65, 1000, 3001])
def test_ragged_sizes(n):
    C = synth.dense_cov(n, 2 * n + 3, seed=n)
    w0 = synth.start_vector(n, n + 1)
    for op in ("min1", "min2"):
        try:
            ref = oracle.mapi(C.astype(np.float64), w0, 30, op=op)
        except oracle.OracleDegenerate:
            # e.g. n = 1 with sign(C) != sign(w0): min2 (eq. 4) is zero, so is the normaliser
            with pytest.raises(mp.MapiError) as ei:
                mp.mapi_solve(to_dev(C), to_dev(w0), max_iters=30, op=op)
            assert ei.value.status == 4
            continue
        w, info = mp.mapi_solve(to_dev(C), to_dev(w0), max_iters=30, op=op)
        assert rel_l1(w.cpu().numpy(), ref.w) <= TOL, op
    b, _ = mp.rpi_solve(to_dev(C), to_dev(w0), max_iters=30)
    assert rel_l1(b.cpu().numpy(), oracle.rpi(C.astype(np.float64), w0, 30).w) <= TOL


def test_zero_iterations_returns_start():
    C = synth.dense_cov(40, 80, seed=1)
    w0 = synth.start_vector(40, 2)
    w, info = mp.mapi_solve(to_dev(C), to_dev(w0), max_iters=0)
    np.testing.assert_array_equal(w.cpu().numpy(), w0)
    assert info["iters"] == 0


def test_degenerate_matrix_is_reported():
    A = np.zeros((64, 64), np.float32)
    with pytest.raises(mp.MapiError) as ei:
        mp.mapi_solve(to_dev(A), to_dev(synth.start_vector(64, 1)), max_iters=5)
    assert ei.value.status == 4


def test_final_l2_and_alias():
    C = synth.dense_cov(128, 300, seed=3)
    w0 = synth.start_vector(128, 4)
    wd = to_dev(w0)
    w, _ = mp.mapi_solve(to_dev(C), wd, max_iters=15, final_l2=True, w_out=wd)
    ref = oracle.mapi(C.astype(np.float64), w0, 15, final_l2=True)
    assert rel_l1(wd.cpu().numpy(), ref.w) <= TOL
    assert abs(np.linalg.norm(wd.cpu().numpy().astype(np.float64)) - 1) < 1e-6


def test_diamond_proposition1_on_gpu():
    rng = np.random.default_rng(10)
    A = rng.uniform(0.1, 2.0, size=(200, 200)).astype(np.float32)
    w0 = rng.uniform(0.1, 1.0, size=200).astype(np.float32)
    row = 1.0 + np.abs(A.astype(np.float64)).sum(axis=1)
    target = row / row.sum()
    w, _ = mp.mapi_solve(to_dev(A), to_dev(w0), max_iters=2, op="diamond")
    assert rel_l1(w.cpu().numpy(), target) <= 1e-6


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_reduced_storage_solve_matches_oracle_on_stored_matrix(dtype):
    C = synth.dense_cov(512, 1024, seed=31)
    w0 = synth.start_vector(512, 32)
    q, s = mp.mapi_quantize(to_dev(C), dtype)
    if dtype == "bf16":
        Aref = oracle.bf16_decode(oracle.bf16_encode(C))
    else:
        qo, so = oracle.fp8_rows_quantize(C)
        Aref = oracle.fp8_rows_dequantize(qo, so)
    for T in (1, 50):
        w, _ = mp.mapi_solve(q, to_dev(w0), max_iters=T, row_scale=s)
        ref = oracle.mapi(Aref.astype(np.float64), w0, T)
        e, c = report(f"mapi {dtype} T={T} vs oracle on stored matrix", w.cpu().numpy(), ref.w)
        assert e <= TOL and c > COS
        full = oracle.mapi(C.astype(np.float64), w0, T)
        report(f"mapi {dtype} T={T} vs oracle on float32 matrix (reported)", w.cpu().numpy(), full.w)
        b, _ = mp.rpi_solve(q, to_dev(w0), max_iters=T, row_scale=s)
        ref_b = oracle.rpi(Aref.astype(np.float64), w0, T)
        assert rel_l1(b.cpu().numpy(), ref_b.w) <= TOL


def test_timing_counts_product_launches():
    # n = 300: one product launch per iteration; n = 256 (float32): the whole solve is one launch
    ctx = mp.Context()
    for n, launches in ((300, 9), (256, 1)):
        C = synth.dense_cov(n, 512, seed=5)
        ctx.timing(True)
        ctx.timing_reset()
        mp.mapi_solve(to_dev(C), to_dev(synth.start_vector(n, 6)), max_iters=9, ctx=ctx)
        ms, count = ctx.timing_get("mavp")
        ctx.timing(False)
        assert count == launches and ms > 0, n


def test_full_size_n16384_sampled_rows_and_iterates():
    # the n = 16384 workload (C = X X^T / 32768), float32 storage, as the benchmark runs it
    n = 16384
    print("[case] full n=16384 generate", flush=True)
    C = synth.dense_cov(n, 32768, seed=2024, device="cuda")
    w0 = synth.start_vector(n, 2025)
    wd = to_dev(w0)
    y = mp.mapi_mavp(C, wd).cpu().numpy()
    Ch = C.cpu().numpy()
    rng = np.random.default_rng(0)
    rows = np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)])
    for i in rows:
        terms = oracle.term_min1(Ch[i], w0)
        assert abs(y[i] - terms.sum()) <= TOL * np.abs(terms).sum()
    print("[case] full n=16384 T=3 vs oracle", flush=True)
    w, _ = mp.mapi_solve(C, wd, max_iters=3)
    ref = oracle.mapi(Ch.astype(np.float64), w0, 3)
    e, c = report("mapi n=16384 T=3", w.cpu().numpy(), ref.w)
    assert e <= TOL and c > COS
    for dtype in ("bf16", "fp8"):
        q, s = mp.mapi_quantize(C, dtype)
        qh = q.cpu().numpy()
        y = mp.mapi_mavp(q, wd, row_scale=s).cpu().numpy()
        for i in rows[:16]:
            if dtype == "bf16":
                qi = oracle.bf16_encode(Ch[i])
                np.testing.assert_array_equal(qh[i].view(np.uint16), qi)
                ai = oracle.bf16_decode(qi)
            else:
                qi, si = oracle.fp8_rows_quantize(Ch[i][None, :])
                np.testing.assert_array_equal(qh[i], qi[0])
                assert s[i].item() == si[0]
                ai = oracle.fp8_rows_dequantize(qi, si)[0]
            terms = oracle.term_min1(ai, w0)
            assert abs(y[i] - terms.sum()) <= TOL * np.abs(terms).sum()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("m,n", [(301, 2061), (67, 1000)])
def test_every_launch_shape_gives_the_same_product(dtype, m, n):
    # Each row's sum is formed by one wave in a fixed lane order whatever the launch shape, and
    # the FP8 sign-word staging (w_in_lds 2) flips signs exactly, so y is bitwise shape-independent.
    # n = 1000 leaves a partial group of 64 vectors in the LDS order (62 FP8 vectors, 125 bf16)
    # and a ragged tail; n = 2061 whole FP8 groups with a 13-column tail.
    rng = np.random.default_rng(11)
    A = rng.standard_normal((m, n)).astype(np.float32)
    w = rng.standard_normal(n).astype(np.float32)
    Ad, rs, Aref = _stored(A, dtype)
    wd = to_dev(w)
    ref = oracle.mavp(Aref.astype(np.float64), w.astype(np.float64), "min1")
    first = None
    lds_modes = (0, 1, 2) if dtype == "fp8" else (0, 1)
    for op in ("min1", "dot"):
        first = None
        for rw in (1, 2, 4, 8):
            for waves in (4, 8):
                for unroll in (2, 4):
                    for lds in lds_modes:
                        for nt in (0, 1):
                            shape = dict(rows_per_wave=rw, waves=waves, blocks_per_cu=1 + (rw & 1), unroll=unroll,
                                         w_in_lds=lds, nontemporal=nt)
                            y = torch.full((m,), float("nan"), device="cuda")
                            mp.mapi_mavp_timed(Ad, wd, shape, op=op, reps=1, row_scale=rs, y=y)
                            yh = y.cpu().numpy()
                            if first is None:
                                first = yh
                                if op == "min1":
                                    assert rel_l1(yh, ref) <= TOL
                            else:
                                np.testing.assert_array_equal(yh, first, err_msg=f"{op} {shape}")


def test_sign_word_staging_rejected_for_other_storage():
    A = to_dev(np.ones((8, 8), np.float32))
    w = to_dev(np.ones(8, np.float32))
    shape = dict(rows_per_wave=1, waves=4, blocks_per_cu=1, unroll=2, w_in_lds=2, nontemporal=0)
    with pytest.raises(mp.MapiError):
        mp.mapi_mavp_timed(A, w, shape, reps=1)


def _sec32_matrix(D, seed):
    # the Sec. 3.2 spectrum: C = V diag(1, 0.9, ..., 0.9) V^T = 0.9 I + 0.1 v v^T, top eigenvector v
    v = synth.start_vector(D, seed).astype(np.float64)
    return (0.9 * np.eye(D) + 0.1 * np.outer(v, v)).astype(np.float32), v


def test_hybrid_matches_chained_calls_and_oracle():
    D = 300
    C, v = _sec32_matrix(D, 21)
    w0 = synth.start_vector(D, 22)
    Cd, wd = to_dev(C), to_dev(w0)
    w, im, ir = mp.mapi_hybrid_solve(Cd, wd, mapi_iters=40, mapi_tol=1e-7, rpi_iters=60, rpi_tol=1e-7)
    assert im["iters"] >= 1 and ir["iters"] >= 1
    # the same as mapi_solve (final l2) followed by rpi_solve
    m1, i1 = mp.mapi_solve(Cd, wd, max_iters=40, tol=1e-7, final_l2=True)
    r1, i2 = mp.rpi_solve(Cd, m1, max_iters=60, tol=1e-7)
    assert (i1["iters"], i2["iters"]) == (im["iters"], ir["iters"])
    np.testing.assert_array_equal(w.cpu().numpy(), r1.cpu().numpy())
    # parity with the oracle at the GPU's iteration counts
    m, r = oracle.hybrid(C.astype(np.float64), w0, im["iters"], ir["iters"])
    e, c = report("hybrid D=300", w.cpu().numpy(), r.w)
    assert e <= TOL and c > COS
    cos = abs(float(r.w @ v)) / np.linalg.norm(r.w)
    assert 1 - cos * cos < 1e-9


def test_hybrid_zero_mapi_iterations_is_rpi():
    D = 257
    C, _ = _sec32_matrix(D, 23)
    w0 = synth.start_vector(D, 24)
    w, im, ir = mp.mapi_hybrid_solve(to_dev(C), to_dev(w0), mapi_iters=0, rpi_iters=30)
    b, _ = mp.rpi_solve(to_dev(C), to_dev(w0 / np.float32(np.linalg.norm(w0))), max_iters=30)
    assert im["iters"] == 0 and ir["iters"] == 30
    np.testing.assert_array_equal(w.cpu().numpy(), b.cpu().numpy())


def test_fp8_mixed_power_of_two_and_general_scales():
    # rows with power-of-two scales take the scaled-conversion decode, others the multiply;
    # both give fl32(s * decode(q)), in every launch shape (row groups may mix the two kinds)
    rng = np.random.default_rng(17)
    m, n = 203, 777
    q = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    q[(q & 0x7F) == 0x7F] = 0                      # no NaN codes
    s = np.where(np.arange(m) % 3 == 0, np.float32(0.6), np.float32(2.0) ** rng.integers(-8, 8, m)).astype(np.float32)
    Aref = oracle.fp8_rows_dequantize(q, s)
    w = rng.standard_normal(n).astype(np.float32)
    ref = oracle.mavp(Aref.astype(np.float64), w.astype(np.float64), "min1")
    qd, sd, wd = to_dev(q), to_dev(s), to_dev(w)
    first = None
    for rw in (1, 2, 4):
        shape = dict(rows_per_wave=rw, waves=4, blocks_per_cu=1, unroll=2, w_in_lds=1, nontemporal=0)
        y = torch.full((m,), float("nan"), device="cuda")
        mp.mapi_mavp_timed(qd, wd, shape, reps=1, row_scale=sd, y=y)
        yh = y.cpu().numpy()
        if first is None:
            first = yh
            terms = np.abs(Aref).sum(axis=1)       # bound scale per row
            assert (np.abs(yh - ref) <= TOL * np.maximum(terms, 1e-30)).all()
        else:
            np.testing.assert_array_equal(yh, first)


def test_read_reference_times_and_rejects_bad_sizes():
    x = torch.ones(1 << 20, dtype=torch.float32, device="cuda")
    ms = mp.mapi_read_reference(x, reps=3)
    assert 0.0 < ms < 100.0
    with pytest.raises(mp.MapiError):
        mp.mapi_read_reference(x[1:], reps=1)           # 4-byte offset: not 16-byte aligned
    with pytest.raises(mp.MapiError):
        mp.mapi_read_reference(x, reps=0)


def _pair_shapes(dtype):
    """Launch shapes that differ only in the staging of w: with w in LDS each product forms its
    own iterate and residual partials and advances the stop rule one launch late; with w read
    from global memory a normalisation kernel follows every product.  Same grid, so the same
    normaliser partials and the same bits of every iterate."""
    base = dict(rows_per_wave=2, waves=8, blocks_per_cu=2, unroll=2, nontemporal=1)
    fused = [dict(base, w_in_lds=l) for l in ((1, 2) if dtype == "fp8" else (1,))]
    return fused, dict(base, w_in_lds=0)


@pytest.mark.parametrize("n", [517, 1003])
@pytest.mark.parametrize("meth", ["mapi", "rpi"])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_stop_rule_in_the_product_matches_the_kernel_pair(dtype, meth, n):
    # fixed iteration counts and tolerance stops: iterates, normalisers and iteration counts are
    # the same bits on both paths; a residual that stopped the solve was summed inside the next
    # product on one path and by the normalisation kernel on the other (float64, another order).
    # n = 517 and 1003 leave ragged tails for every storage type.
    print(f"[case] stop rule in the product {dtype} {meth} n={n}", flush=True)
    A32, _, _ = synth.planted_symmetric(n, [0.4], seed=n)
    Ad, rs, Aref = _stored(A32, dtype)
    w0h = synth.start_vector(n, n + 1)
    w0 = to_dev(w0h)
    code = {"f32": mp.MAPI_F32, "bf16": mp.MAPI_BF16, "fp8": mp.MAPI_FP8_E4M3}[dtype]
    fn = mp.mapi_solve if meth == "mapi" else mp.rpi_solve
    fused, pair = _pair_shapes(dtype)
    for T, tol in ((13, 0.0), (500, 1e-5)):
        mp.mapi_tuning_set(code, n, n, pair)
        wb, ib = fn(Ad, w0, max_iters=T, tol=tol, check_every=5, row_scale=rs)
        for shape in fused:
            mp.mapi_tuning_set(code, n, n, shape)
            wa, ia = fn(Ad, w0, max_iters=T, tol=tol, check_every=5, row_scale=rs)
            np.testing.assert_array_equal(wa.cpu().numpy(), wb.cpu().numpy())
            assert ia["iters"] == ib["iters"] and ia["converged"] == ib["converged"], (ia, ib)
            assert ia["norm"] == ib["norm"]
            assert ia["residual"] == pytest.approx(ib["residual"], rel=1e-12, abs=0)
        if tol == 0.0:
            assert ia["iters"] == T and ia["residual"] == ib["residual"]
        else:
            assert ia["converged"] and ia["residual"] < tol and ia["iters"] < T
        t = ia["iters"]
        ref = (oracle.mapi if meth == "mapi" else oracle.rpi)(Aref.astype(np.float64), w0h.astype(np.float64), t)
        e = rel_l1(wa.cpu().numpy(), ref.w)
        assert e <= TOL
        # |r_gpu - r_oracle| <= ||w_t err||_1 + ||w_{t-1} err||_1 (triangle inequality); the
        # iterate error measured at t, with a factor 4 for the previous iterate and slack
        bound = 4 * e * np.abs(ref.w).sum() + 1e-3 * ref.residuals[-1] + 1e-9
        assert abs(ia["residual"] - ref.residuals[-1]) <= bound
        if tol > 0.0:
            stop = (oracle.mapi if meth == "mapi" else oracle.rpi)(Aref.astype(np.float64), w0h.astype(np.float64),
                                                                    T, tol=tol)
            assert abs(stop.iters - t) <= 2


@pytest.mark.parametrize("n", [512, 1024, 4096])
@pytest.mark.parametrize("meth", ["mapi", "rpi"])
def test_stop_rule_in_the_product_exact_residuals(meth, n):
    # A constant positive matrix and a positive start, both dyadic (so every row sum is exact,
    # whatever order the kernel adds its terms in, and all rows' sums are equal): the first
    # iterate is the constant vector (1/n for MAPI, 1/sqrt(n) for RPI, exact for these n) and
    # every later residual is exactly 0.  So the stop iteration of each rule is known exactly:
    # a zero tolerance never converges;
    # tol 1e-300 stops at iteration 2; the stall rule with k = 3 stops at 2 + 3 = 5 (iteration 2
    # sets the smallest residual, 0, and three iterations do not beat it).  The lagged decision
    # is taken by the next product (T > t + 1), by the last normalisation (T = t + 1) or not at
    # all (T <= t).
    print(f"[case] exact stop rule {meth} n={n}", flush=True)
    A = to_dev(np.full((n, n), 0.75, np.float32))
    w0h = (np.random.default_rng(n).integers(7, 65, n) / 64.0).astype(np.float32)
    w0 = to_dev(w0h)
    fn = mp.mapi_solve if meth == "mapi" else mp.rpi_solve
    const = 1.0 / n if meth == "mapi" else 1.0 / np.sqrt(n)
    fused, pair = _pair_shapes("f32")
    cases = [  # T, tol, stall -> iters, converged
        (7, 0.0, 0, 7, False), (9, 1e-300, 0, 2, True), (2, 1e-300, 0, 2, True), (3, 1e-300, 0, 2, True),
        (1, 1e-300, 0, 1, False), (12, 0.0, 3, 5, False), (5, 0.0, 3, 5, False), (6, 0.0, 3, 5, False),
        (4, 0.0, 3, 4, False)]
    for shape in fused + [pair]:
        mp.mapi_tuning_set(mp.MAPI_F32, n, n, shape)
        for T, tol, stall, iters, conv in cases:
            w, info = fn(A, w0, max_iters=T, tol=tol, stall_iters=stall, check_every=1 + T % 3)
            assert info["iters"] == iters and info["converged"] == conv, (shape, T, tol, stall, info)
            if iters >= 2:
                assert info["residual"] == 0.0
                np.testing.assert_array_equal(w.cpu().numpy(), np.full(n, const, np.float32))
            ref = (oracle.mapi if meth == "mapi" else oracle.rpi)(np.full((n, n), 0.75, np.float64),
                                                                    w0h.astype(np.float64), iters)
            assert rel_l1(w.cpu().numpy(), ref.w) <= TOL
            assert info["norm"] == pytest.approx(ref.norms[-1], rel=1e-6)


def test_degenerate_normaliser_in_the_product_is_reported():
    # the zero matrix: the first normaliser is zero whether the product or the kernel forms it
    n = 96
    mp.mapi_tuning_set(mp.MAPI_F32, n, n, dict(rows_per_wave=1, waves=4, blocks_per_cu=1, unroll=2, w_in_lds=1,
                                               nontemporal=0))
    for tol in (0.0, 1e-300):
        with pytest.raises(mp.MapiError) as ei:
            mp.mapi_solve(to_dev(np.zeros((n, n), np.float32)), to_dev(synth.start_vector(n, 1)), max_iters=5, tol=tol)
        assert ei.value.status == 4 and "after 0 iterations" in str(ei.value)


@pytest.mark.parametrize("n", [1, 3, 17, 64])
@pytest.mark.parametrize("T", [1, 2, 3])
def test_normalisation_in_the_product_edge_cases(n, T):
    # tiny sizes (one vector or only a ragged tail), one and two iterations (no product that
    # forms the iterate, or exactly one), final l2 and an output that aliases the start vector:
    # the fixed-iteration solve with w staged in LDS (the product forms the iterate) equals the one
    # with w read from global memory (normalisation kernel after every product; same row sums).
    # (A tolerance cannot force the second path here: at n = 1 the iterate is exactly +-1 after one
    # step, so any positive tolerance stops the solve on a zero residual.)
    print(f"[case] fused normalisation edge n={n} T={T}", flush=True)
    rng = np.random.default_rng(n * 10 + T)
    A = to_dev((rng.standard_normal((n, n)) + 3.0).astype(np.float32))
    w0h = rng.uniform(0.5, 1.0, n).astype(np.float32)
    shape = dict(rows_per_wave=1, waves=4, blocks_per_cu=1, unroll=2, nontemporal=0)
    for final_l2 in (False, True):
        res = []
        for lds in (1, 0):
            mp.mapi_tuning_set(mp.MAPI_F32, n, n, dict(shape, w_in_lds=lds))
            res.append(mp.mapi_solve(A, to_dev(w0h), max_iters=T, final_l2=final_l2))
        (wa, ia), (wb, ib) = res
        np.testing.assert_array_equal(wa.cpu().numpy(), wb.cpu().numpy())
        assert ia["iters"] == ib["iters"] == T and ia["norm"] == ib["norm"] and ia["residual"] == ib["residual"]
        mp.mapi_tuning_set(mp.MAPI_F32, n, n, dict(shape, w_in_lds=1))
        alias = to_dev(w0h)
        wc, _ = mp.mapi_solve(A, alias, max_iters=T, final_l2=final_l2, w_out=alias)
        np.testing.assert_array_equal(wc.cpu().numpy(), wa.cpu().numpy())
