"""GPU parity of the factored operator X (+) (X^T (+) w) (mapi_factored_solve; not a method of the
paper) against the FP64 oracle (oracle.factored_mapi), on ragged shapes, both min forms, a padded
row pitch, the sign-matrix closed form, and the full PCA size.  Tolerance: relative l1 <= 1e-5
and cosine > 1 - 1e-6 at the same iteration count."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel_l1, report, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5
COS = 1 - 1e-6


@pytest.mark.parametrize("op", ["min1", "min2"])
@pytest.mark.parametrize("D,N,T", [(64, 300, 12), (200, 1001, 10), (130, 4099, 8), (1, 7, 3), (300, 2, 4),
                                   (257, 33, 15)])
def test_factored_matches_oracle(D, N, T, op):
    print(f"[case] factored D={D} N={N} T={T} {op}", flush=True)
    X = synth.pca_data(D, N, seed=D * 7 + N)
    w0 = synth.start_vector(D, D + N)
    try:
        ref = oracle.factored_mapi(X.astype(np.float64), w0, T, scale=1.0 / N, op=op)
    except oracle.OracleDegenerate:
        # min2 keeps only equal-sign terms: with one row, w's sign can leave no term (a zero
        # normaliser), which the GPU reports as degenerate too
        with pytest.raises(mp.MapiError) as ei:
            mp.mapi_factored_solve(to_dev(X), to_dev(w0), max_iters=T, op=op)
        assert ei.value.status == 4
        return
    w, info = mp.mapi_factored_solve(to_dev(X), to_dev(w0), max_iters=T, op=op)
    assert info["iters"] == T and info["status"] == "OK"
    e, c = report(f"factored D={D} N={N} {op}", w.cpu().numpy(), ref.w)
    assert e <= TOL and c > COS
    assert info["norm"] == pytest.approx(ref.norms[-1], rel=1e-5)


def test_factored_tolerance_stop_and_padded_rows():
    # a tolerance stop compared at the GPU's iteration count; X as a view of a buffer whose row
    # padding holds NaN (a read past column N would poison the result): same bits as contiguous
    D, N, ld = 96, 501, 512
    X = synth.pca_data(D, N, seed=5)
    w0 = synth.start_vector(D, 6)
    buf = torch.full((D, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :N] = torch.from_numpy(X).cuda()
    Xp = buf[:, :N]
    w1, i1 = mp.mapi_factored_solve(Xp, to_dev(w0), max_iters=300, tol=1e-6, check_every=4, stall_iters=10)
    w2, i2 = mp.mapi_factored_solve(to_dev(X), to_dev(w0), max_iters=300, tol=1e-6, check_every=4, stall_iters=10)
    assert i1 == i2
    np.testing.assert_array_equal(w1.cpu().numpy(), w2.cpu().numpy())
    ref = oracle.factored_mapi(X.astype(np.float64), w0, i1["iters"], scale=1.0 / N)
    e, c = report("factored tolerance stop", w1.cpu().numpy(), ref.w)
    assert e <= TOL and c > COS
    print(f"[iters] factored to 1e-6: gpu {i1['iters']} (converged {i1['converged']})", flush=True)


def test_factored_sign_matrix_closed_form_on_gpu():
    # |X_ik| >= 1 and ||w||_1 = 1: each step is l1 power iteration on S S^T, S = sign(X)
    rng = np.random.default_rng(8)
    D, N, T = 48, 700, 30
    X = (rng.uniform(1.0, 3.0, size=(D, N)) * np.where(rng.uniform(size=(D, N)) < 0.55, 1.0, -1.0)).astype(np.float32)
    w0 = np.abs(synth.start_vector(D, 9))
    w0 = (w0 / w0.sum()).astype(np.float32)
    w, info = mp.mapi_factored_solve(to_dev(X), to_dev(w0), max_iters=T)
    S = np.sign(X.astype(np.float64))
    M = S @ S.T
    v = w0.astype(np.float64)
    for _ in range(T):
        y = M @ v
        v = y / np.abs(y).sum()
    assert rel_l1(w.cpu().numpy(), v) <= TOL


def test_factored_argument_checks():
    X = torch.zeros((8, 16), dtype=torch.float32, device="cuda")
    w0 = torch.full((8,), 0.125, dtype=torch.float32, device="cuda")
    with pytest.raises(mp.MapiError) as ei:
        mp.mapi_factored_solve(X, w0, op="dot")
    assert ei.value.status == 6
    with pytest.raises(mp.MapiError) as ei:
        mp.mapi_factored_solve(X, w0, scale=-1.0)
    assert ei.value.status == 1
    # a zero matrix gives a zero normaliser on the first step
    with pytest.raises(mp.MapiError) as ei:
        mp.mapi_factored_solve(X, w0, max_iters=3)
    assert ei.value.status == 4


def test_factored_full_pca_size_three_iterations():
    # the PCA workload's X (4096 x 65536, 1 GiB): three iterations against the FP64 oracle
    D, N, T = 4096, 65536, 3
    print("[case] factored full size: generate", flush=True)
    X, _ = synth.pca_data_device(D, N, 77, "cuda")
    w0 = synth.start_vector(D, 78)
    w, info = mp.mapi_factored_solve(X, to_dev(w0), max_iters=T)
    Xh = X.cpu().numpy().astype(np.float64)
    print("[case] factored full size: oracle", flush=True)
    ref = oracle.factored_mapi(Xh, w0, T, scale=1.0 / N)
    e, c = report("factored 4096 x 65536 T=3", w.cpu().numpy(), ref.w)
    assert e <= TOL and c > COS
