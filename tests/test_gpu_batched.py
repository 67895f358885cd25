"""GPU parity of the persistent batched solver: each instance against the FP64 oracle,
alone versus in a mix (bitwise), and against the one-at-a-time path."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel_l1, report, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5


@pytest.mark.parametrize("n", [1, 5, 64, 300, 1500])
def test_generator_matches_definition(n):
    A, w0 = mp.mapi_generate_dense(n, 12345 + n)
    Ar, wr = synth.generated_dense(n, 12345 + n)
    np.testing.assert_array_equal(A.cpu().numpy(), Ar)
    np.testing.assert_array_equal(w0.cpu().numpy(), wr)


def test_batched_dense_user_matrices_match_oracle():
    cases = []
    specs = [(256, "f32", "mapi"), (3000, "f32", "mapi"), (3000, "f32", "rpi"), (2000, "bf16", "mapi"),
             (1200, "fp8", "rpi"), (700, "f32", "rpi"), (1500, "fp8", "mapi")]
    probs = []
    for k, (n, dt, meth) in enumerate(specs):
        C = synth.dense_cov(n, 2 * n, seed=100 + k)
        w0 = synth.start_vector(n, 200 + k)
        if dt == "f32":
            Ad, rs, Aref = to_dev(C), None, C
        elif dt == "bf16":
            q = oracle.bf16_encode(C)
            Ad, rs, Aref = to_dev(q.view(np.int16)), None, oracle.bf16_decode(q)
        else:
            q, s = oracle.fp8_rows_quantize(C)
            Ad, rs, Aref = to_dev(q), to_dev(s), oracle.fp8_rows_dequantize(q, s)
        probs.append(mp.problem_dense(Ad, meth, w0=to_dev(w0), row_scale=rs, max_iters=30))
        cases.append((Aref, w0, meth, dt, n))
    infos = mp.mapi_solve_batched(probs)
    for p, info, (Aref, w0, meth, dt, n) in zip(probs, infos, cases):
        assert info["iters"] == 30 and info["status"] == "OK"
        fn = oracle.mapi if meth == "mapi" else oracle.rpi
        ref = fn(Aref.astype(np.float64), w0, 30)
        e, _ = report(f"batched {meth} {dt} n={n}", p.out.cpu().numpy(), ref.w)
        assert e <= TOL


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batched_generated_to_tolerance_match_oracle(dtype):
    specs = [(100, "mapi"), (100, "rpi"), (2500, "mapi"), (2500, "rpi"), (1025, "mapi")]
    probs = [mp.problem_generated(n, 7000 + k, dtype, meth, max_iters=400, tol=1e-6) for k, (n, meth) in enumerate(specs)]
    infos = mp.mapi_solve_batched(probs)
    for k, (p, info, (n, meth)) in enumerate(zip(probs, infos, specs)):
        assert info["status"] == "OK"
        A, w0 = synth.generated_dense(n, 7000 + k)
        if dtype == "bf16":
            A = oracle.bf16_decode(oracle.bf16_encode(A))
        fn = oracle.mapi if meth == "mapi" else oracle.rpi
        ref = fn(A.astype(np.float64), w0, info["iters"])
        e, _ = report(f"batched generated {dtype} {meth} n={n} iters={info['iters']} conv={info['converged']}",
                      p.out.cpu().numpy(), ref.w)
        assert e <= TOL


def test_batched_pagerank_matches_oracle():
    probs, graphs = [], []
    for k, (n, meth) in enumerate([(500, "mapi"), (500, "rpi"), (20000, "mapi"), (20000, "rpi"), (9000, "mapi")]):
        g = synth.powerlaw_graph(n, seed=300 + k)
        rp, col, val = (torch.from_numpy(g[x]).cuda() for x in ("row_ptr", "col", "val"))
        probs.append(mp.problem_csr(rp, col, val, 0.85, meth, max_iters=12))
        graphs.append((g, meth))
    infos = mp.mapi_solve_batched(probs)
    for p, info, (g, meth) in zip(probs, infos, graphs):
        assert info["iters"] == 12
        ref = oracle.pagerank(g["n"], g["row_ptr"], g["col"], g["val"], 0.85, meth, synth.uniform_start(g["n"]), 12)
        e, _ = report(f"batched pagerank {meth} n={g['n']}", p.out.cpu().numpy(), ref.w)
        assert e <= TOL


def _mix(seed, k):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(k):
        n = int(np.exp(rng.uniform(np.log(64), np.log(4096))))
        probs.append(mp.problem_generated(n, 50000 + seed * 1000 + i, ["f32", "bf16"][i % 2], ["mapi", "rpi"][(i // 2) % 2],
                                          max_iters=200, tol=1e-6))
    return probs


def test_alone_equals_in_mix_bitwise():
    ctx = mp.Context()
    g = synth.powerlaw_graph(5000, seed=4)
    rp, col, val = (torch.from_numpy(g[x]).cuda() for x in ("row_ptr", "col", "val"))
    C = synth.dense_cov(600, 1200, seed=5)

    def targets():
        return [mp.problem_generated(2000, 99, "f32", "mapi", max_iters=200, tol=1e-6),
                mp.problem_generated(800, 98, "bf16", "rpi", max_iters=200, tol=1e-6),
                mp.problem_csr(rp, col, val, 0.85, "mapi", max_iters=50, tol=1e-7),
                mp.problem_dense(to_dev(C), "mapi", w0=to_dev(synth.start_vector(600, 6)), max_iters=60)]
    alone = []
    for p in targets():
        info = mp.mapi_solve_batched([p], ctx=ctx)[0]
        alone.append((p.out.cpu().numpy().copy(), info["iters"]))
    mixed = targets()
    batch = _mix(1, 24)
    batch[3:3] = mixed[:2]
    batch.extend(mixed[2:])
    infos = mp.mapi_solve_batched(batch, ctx=ctx)
    by_id = {id(p): i for i, p in enumerate(batch)}
    for (w_alone, it_alone), p in zip(alone, mixed):
        i = by_id[id(p)]
        assert infos[i]["iters"] == it_alone
        np.testing.assert_array_equal(p.out.cpu().numpy(), w_alone)


def test_batched_matches_one_at_a_time_path():
    for n, dt in ((1500, "f32"), (600, "f32")):
        p = mp.problem_generated(n, 31337, dt, "mapi", max_iters=80)
        mp.mapi_solve_batched([p])
        A, w0 = mp.mapi_generate_dense(n, 31337)
        w, info = mp.mapi_solve(A, w0, max_iters=80)
        assert rel_l1(p.out.cpu().numpy(), w.cpu().numpy()) <= 1e-6


def test_batched_degenerate_instance_is_isolated():
    Z = np.zeros((300, 300), np.float32)
    C = synth.dense_cov(300, 600, seed=8)
    w0 = to_dev(synth.start_vector(300, 9))
    probs = [mp.problem_dense(to_dev(Z), "mapi", w0=w0, max_iters=10),
             mp.problem_dense(to_dev(C), "mapi", w0=w0, max_iters=10),
             mp.problem_generated(3000, 5, "f32", "rpi", max_iters=10)]
    infos = mp.mapi_solve_batched(probs)
    assert infos[0]["status"] == "ERR_DEGENERATE"
    assert infos[1]["status"] == "OK" and infos[1]["iters"] == 10
    assert infos[2]["status"] == "OK" and infos[2]["iters"] == 10
    ref = oracle.mapi(C.astype(np.float64), synth.start_vector(300, 9), 10)
    assert rel_l1(probs[1].out.cpu().numpy(), ref.w) <= TOL


def test_zero_iterations_and_empty_batch():
    assert mp.mapi_solve_batched([]) == []
    p = mp.problem_generated(700, 3, "f32", "mapi", max_iters=0)
    info = mp.mapi_solve_batched([p])[0]
    A, w0 = synth.generated_dense(700, 3)
    assert info["iters"] == 0
    np.testing.assert_array_equal(p.out.cpu().numpy(), w0)


def test_autotune_batched_row_split():
    rows, ms = mp.mapi_autotune_batched(mp.MAPI_F32, 4096, count=16, iters=4)
    # the candidate tile heights: powers of two from 4 to 1024 rows (mapi_batched_rows_set)
    assert rows in (4, 8, 16, 32, 64, 128, 256, 512, 1024) and ms > 0
    assert mp.mapi_batched_rows_get(mp.MAPI_F32, 4096) == rows
    p = mp.problem_generated(4096, 77, "f32", "mapi", max_iters=5)
    mp.mapi_solve_batched([p])
    A, w0 = synth.generated_dense(4096, 77)
    ref = oracle.mapi(A.astype(np.float64), w0, 5)
    assert rel_l1(p.out.cpu().numpy(), ref.w) <= TOL
