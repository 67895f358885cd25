"""GPU parity of the Gram builds (eq. 5 min-covariance, eq. 2 covariance) and top-k PCA with deflation."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import cosine, rel_l1, report, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2110_12065_amd as mp  # noqa: E402

TOL = 1e-5


@pytest.mark.parametrize("op", ["min1", "min2", "dot"])
@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (64, 300), (130, 1000), (200, 4099), (1000, 200)])
def test_gram_dyadic_bitexact(op, shape):
    # (5, 7) and (1000, 200) take one sample chunk (36 tiles of 128 at D = 1000, each written with
    # its mirror by the build kernel); (64, 300), (130, 1000) and (200, 4099) split the samples into
    # 2, 4 and 6 (dot) or 9 (min forms) chunks summed by the reduction kernel
    D, N = shape
    print(f"[case] gram dyadic {op} {shape}", flush=True)
    X = synth.dyadic_matrix(D, N, seed=D * 13 + N)
    A = mp.mapi_mingram(to_dev(X), 0.25, op).cpu().numpy()
    ref = oracle.mingram(X, 0.25, op).astype(np.float32)
    np.testing.assert_array_equal(A, ref)


@pytest.mark.parametrize("op", ["min1", "min2", "dot"])
def test_gram_padded_rows_match_contiguous(op):
    # X as a view of a buffer with row pitch 1008 > N = 1001 whose padding holds NaN: a read
    # past sample N would poison the result; the sums must equal the contiguous build's bits
    D, N, ld = 200, 1001, 1008
    X = synth.pca_data(D, N, seed=9)
    buf = torch.full((D, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :N] = to_dev(X)
    Xp = buf[:, :N]
    assert Xp.stride(0) == ld and not Xp.is_contiguous()
    A = mp.mapi_mingram(Xp, 1.0 / N, op).cpu().numpy()
    B = mp.mapi_mingram(to_dev(X), 1.0 / N, op).cpu().numpy()
    assert np.isfinite(A).all()
    np.testing.assert_array_equal(A, B)


@pytest.mark.parametrize("op", ["min1", "dot"])
def test_gram_random_within_bound(op):
    D, N = 256, 4096
    X = synth.pca_data(D, N, seed=3)
    scale = 1.0 / N
    A = mp.mapi_mingram(to_dev(X), scale, op).cpu().numpy().astype(np.float64)
    ref = oracle.mingram(X, scale, op)
    absum = oracle.mingram(np.abs(X), scale, "min1" if op == "min1" else "dot")
    assert np.all(np.abs(A - ref) <= TOL * absum + 1e-30)
    np.testing.assert_array_equal(A, A.T)
    if op == "min1":
        np.testing.assert_allclose(np.diag(A), scale * np.abs(X.astype(np.float64)).sum(axis=1), rtol=1e-6)


@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_pca_topk_matches_oracle(method):
    D, N, k, T = 256, 4096, 4, 40
    X = synth.pca_data(D, N, seed=5)
    W0 = synth.start_vectors(D, k, seed=6)
    P, infos = mp.mapi_pca_topk(to_dev(X), k, to_dev(W0), method=method, max_iters=T)
    P = P.cpu().numpy().astype(np.float64)
    Pr, res = oracle.pca_topk(X, k, W0, method=method, T=T)
    for i in range(k):
        assert infos[i]["iters"] == T
        e, c = report(f"pca {method} vector {i}", P[:, i], Pr[:, i])
        assert e <= TOL and c > 1 - 1e-6
    np.testing.assert_allclose(P.T @ P, np.eye(k), atol=1e-6)


@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_pca_topk_seeded_starts(method):
    # W0 = None: vector i starts from the generated start vector of seed i, the same bits as
    # passing those vectors (written by the host generator) explicitly; and against the oracle
    D, N, k, T = 200, 1500, 3, 25
    X = synth.pca_data(D, N, seed=11)
    W0 = np.stack([synth.generated_start(D, i) for i in range(k)], axis=1)
    Pn, inn = mp.mapi_pca_topk(to_dev(X), k, None, method=method, max_iters=T)
    Pe, ine = mp.mapi_pca_topk(to_dev(X), k, to_dev(W0), method=method, max_iters=T)
    np.testing.assert_array_equal(Pn.cpu().numpy(), Pe.cpu().numpy())
    assert [i["iters"] for i in inn] == [i["iters"] for i in ine] == [T] * k
    Pr, _ = oracle.pca_topk(X, k, W0, method=method, T=T)
    P = Pn.cpu().numpy().astype(np.float64)
    for i in range(k):
        e, c = report(f"pca seeded {method} vector {i}", P[:, i], Pr[:, i])
        assert e <= TOL and c > 1 - 1e-6


def test_pca_topk_tolerance_per_vector():
    D, N, k = 128, 2048, 3
    X = synth.pca_data(D, N, seed=7)
    W0 = synth.start_vectors(D, k, seed=8)
    P, infos = mp.mapi_pca_topk(to_dev(X), k, to_dev(W0), method="rpi", max_iters=2000, tol=1e-6, check_every=8)
    A = oracle.covariance(X, 1.0 / N)
    lam, V = np.linalg.eigh(A)
    P = P.cpu().numpy()
    for i in range(k):
        assert infos[i]["converged"]
        assert abs(cosine(P[:, i], V[:, -1 - i])) > 1 - 1e-5


def test_gram_min1_xor_form_same_bits(monkeypatch):
    # the three-instruction min1 term (sign-bit flip, med3, add) builds the same matrix, bit for
    # bit, as the two-instruction one (med3, FMA by +-1); with the sample chunks split (D = 300,
    # N = 5000) and whole
    for D, N in ((300, 5000), (130, 700)):
        X = synth.pca_data(D, N, seed=D + N)
        A = mp.mapi_mingram(to_dev(X), 1.0 / N, "min1").cpu().numpy()
        monkeypatch.setenv("MAPI_MIN1_FORM", "xor")
        B = mp.mapi_mingram(to_dev(X), 1.0 / N, "min1").cpu().numpy()
        monkeypatch.delenv("MAPI_MIN1_FORM")
        np.testing.assert_array_equal(A, B)


def test_full_size_gram_sampled_entries():
    # the PCA workload: D = 4096 coordinates x N = 65536 samples, 16 factors + noise + 5 % Laplace outliers
    D, N = 4096, 65536
    print("[case] full PCA generate", flush=True)
    X = synth.pca_data(D, N, seed=77)
    Xd = to_dev(X)
    print("[case] full PCA gram", flush=True)
    A = mp.mapi_mingram(Xd, 1.0 / N, "min1").cpu().numpy()
    np.testing.assert_array_equal(A, A.T)
    rng = np.random.default_rng(1)
    pairs = [(0, 0), (D - 1, D - 1), (0, D - 1), (63, 64), (64, 63)] + [tuple(p) for p in rng.integers(0, D, (40, 2))]
    for i, j in pairs:
        ref = oracle.mingram_entry(X, i, j, 1.0 / N)
        bound = oracle.mingram_entry(np.abs(X[[i]]), 0, 0, 1.0 / N) if i == j else \
            float(np.sum(np.minimum(np.abs(X[i].astype(np.float64)), np.abs(X[j].astype(np.float64)))) / N)
        assert abs(A[i, j] - ref) <= TOL * bound, (i, j)
    print("[case] full PCA covariance (matrix cores, 8 sample chunks)", flush=True)
    del A
    C = mp.mapi_mingram(Xd, 1.0 / N, "dot").cpu().numpy()
    np.testing.assert_array_equal(C, C.T)
    for i, j in pairs:
        ref = oracle.mingram_entry(X, i, j, 1.0 / N, "dot")
        bound = float(np.sum(np.abs(X[i].astype(np.float64) * X[j].astype(np.float64))) / N)
        assert abs(C[i, j] - ref) <= TOL * bound, (i, j)
    del C
    print("[case] full PCA top-8", flush=True)
    W0 = synth.start_vectors(D, 8, seed=78)
    P, infos = mp.mapi_pca_topk(Xd, 8, to_dev(W0), method="mapi", max_iters=50)
    P = P.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(P.T @ P, np.eye(8), atol=1e-6)
    assert all(i["iters"] == 50 for i in infos)


@pytest.mark.parametrize("method", ["mapi", "rpi"])
def test_full_size_pca_top8_matches_oracle_on_the_gpu_built_matrix(method):
    # the PCA workload (D = 4096, N = 65536, top 8, device-generated data) with a tolerance of
    # 1e-6 and at most 30 iterations per vector; the FP64 oracle runs the deflation chain on the
    # same matrix (the GPU build, promoted) for each vector's GPU iteration count
    D, N, k = 4096, 65536, 8
    print(f"[case] full PCA top-8 {method}: generate", flush=True)
    X, _ = synth.pca_data_device(D, N, seed=77, device="cuda")
    op = "min1" if method == "mapi" else "dot"
    A = mp.mapi_mingram(X, 1.0 / N, op).cpu().numpy().astype(np.float64)
    W0 = synth.start_vectors(D, k, seed=78)
    print(f"[case] full PCA top-8 {method}: GPU", flush=True)
    P, infos = mp.mapi_pca_topk(X, k, to_dev(W0), method=method, max_iters=30, tol=1e-6, check_every=4)
    del X
    P = P.cpu().numpy().astype(np.float64)
    counts = [i["iters"] for i in infos]
    print(f"[case] full PCA top-8 {method}: oracle at iterations {counts}", flush=True)
    Pr, res = oracle.pca_topk(np.zeros((D, 1), np.float32), k, W0, method=method, T=counts, A=A)
    for i in range(k):
        assert res[i].iters == counts[i]
        e, c = report(f"full pca {method} vector {i} ({counts[i]} iterations)", P[:, i], Pr[:, i])
        assert e <= TOL and c > 1 - 1e-6
        if infos[i]["converged"]:
            assert res[i].residuals[-1] < 2e-6       # the oracle's residual at the GPU's stop
    np.testing.assert_allclose(P.T @ P, np.eye(k), atol=1e-6)
