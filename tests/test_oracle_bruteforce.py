"""Exact rational brute force of the MAVP product and of MAPI on tiny systems (no GPU).

The min1 product of eq. (3) uses only signs, minima and additions, and Algorithm 1's
normaliser and the residual ||w_t - w_{t-1}||_1 are sums of absolute values followed by a
division, so on rational inputs every quantity of the iteration is rational.
``fractions.Fraction`` therefore gives the exact iterates, normalisers and residuals for
n <= 8 and t <= 5 (the optional l2 step of Algorithm 1 needs a square root and is left
out).  The inputs are dyadic (k / 8), so the float64 oracle starts from exactly the same
numbers; its only error is the rounding of its own arithmetic, a few units of float64
precision per step.

Every quantity the oracle returns is compared with the exact one at a bound far below the
size of a plausible mistake: the tests also show, on the same inputs, that an l2 or max-norm
residual, a transposed product, a dropped term or a missing absolute value in the
normaliser would be caught.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

REL = 1e-12      # float64 arithmetic over <= 5 steps of <= 8-term sums
N_CASES = 40


# ---------------------------------------------------------------- exact arithmetic
def sgn(x):
    return (x > 0) - (x < 0)


def min1_exact(a, b):
    """eq. (3): sign(a b) min(|a|, |b|), in rationals."""
    return sgn(a) * sgn(b) * min(abs(a), abs(b))


def min2_exact(a, b):
    """eq. (4): 1(sign a = sign b) min(|a|, |b|)."""
    return min(abs(a), abs(b)) if sgn(a) == sgn(b) else Fr(0)


def mavp_exact(A, w, term=min1_exact):
    """Row i of A against w (the matrix extension of Sec. 2.1)."""
    return [sum((term(A[i][j], w[j]) for j in range(len(w))), Fr(0)) for i in range(len(A))]


def matvec_exact(A, w):
    return [sum((A[i][j] * w[j] for j in range(len(w))), Fr(0)) for i in range(len(A))]


def power_exact(step, w0, T):
    """Algorithm 1 with the l1 normaliser (eq. 6): the exact iterates, normalisers and
    l1 residuals of T steps (stops early, returning what it has, if a normaliser is 0)."""
    w = list(w0)
    ws, nus, rs = [], [], []
    for _ in range(T):
        y = step(w)
        nu = sum((abs(v) for v in y), Fr(0))
        if nu == 0:
            break
        w_new = [v / nu for v in y]
        rs.append(sum((abs(a - b) for a, b in zip(w_new, w)), Fr(0)))
        nus.append(nu)
        ws.append(w_new)
        w = w_new
    return ws, nus, rs


def dyadic_case(rng, n, zeros=True):
    """A (n x n) and w0 with entries k/8, |k| <= 16 (exact in float64 and float32)."""
    A = rng.integers(-16, 17, size=(n, n))
    w0 = rng.integers(-16, 17, size=n)
    if not zeros:
        A[A == 0] = 3
        w0[w0 == 0] = -5
    if not w0.any():
        w0[0] = 7
    return A / 8.0, w0 / 8.0


def to_fr(M):
    M = np.asarray(M, dtype=np.float64)
    if M.ndim == 1:
        return [Fr(float(v)) for v in M]
    return [[Fr(float(v)) for v in row] for row in M]


def close(x, exact, scale):
    return abs(float(x) - float(exact)) <= REL * scale


def cases():
    rng = np.random.default_rng(20211022)
    out = []
    for c in range(N_CASES):
        n = 1 + c % 8
        out.append((n, *dyadic_case(rng, n, zeros=c % 3 != 0)))
    return out


# ---------------------------------------------------------------- product
@pytest.mark.parametrize("op,term", [("min1", min1_exact), ("min2", min2_exact)])
def test_mavp_equals_exact_rational_product(op, term):
    for n, A, w in cases():
        exact = mavp_exact(to_fr(A), to_fr(w), term)
        y = oracle.mavp(A, w, op)
        # every partial sum of k/8 terms is exact in float64: the oracle must agree exactly
        assert [Fr(float(v)) for v in y] == exact, (n, op)


def test_mavp_pin_catches_transposed_and_dropped_terms():
    caught_t = caught_d = 0
    for n, A, w in cases():
        exact = mavp_exact(to_fr(A), to_fr(w))
        yt = mavp_exact(to_fr(A.T), to_fr(w))
        caught_t += yt != exact
        y_drop = [sum((min1_exact(Fr(float(A[i, j])), Fr(float(w[j]))) for j in range(1, n)), Fr(0))
                  for i in range(n)]
        caught_d += y_drop != exact
    assert caught_t >= N_CASES // 2 and caught_d >= N_CASES // 2


# ---------------------------------------------------------------- MAPI (Algorithm 1)
def test_mapi_iterates_normalisers_and_l1_residuals_are_exact():
    checked = 0
    for n, A, w0 in cases():
        ws, nus, rs = power_exact(lambda w: mavp_exact(to_fr(A), w), to_fr(w0), 5)
        if len(ws) < 5:
            with pytest.raises(oracle.OracleDegenerate):
                oracle.mapi(A, w0, 5)
            continue
        res = oracle.mapi(A, w0, 5)
        assert res.iters == 5 and len(res.norms) == 5 and len(res.residuals) == 5
        for t in range(5):
            assert close(res.norms[t], nus[t], float(nus[t])), (n, t, "nu")
            assert close(res.residuals[t], rs[t], 1.0), (n, t, "r")
        for v, e in zip(res.w, ws[-1]):
            assert close(v, e, 1.0), (n, "w")
        checked += 1
    assert checked >= N_CASES // 2


def test_mapi_stops_at_the_first_exact_residual_below_tol():
    done = 0
    for n, A, w0 in cases():
        ws, nus, rs = power_exact(lambda w: mavp_exact(to_fr(A), w), to_fr(w0), 5)
        if len(ws) < 5 or n < 2:
            continue
        # a tolerance half-way (geometrically) between two exact residual values, so no
        # rounding can move the stop
        vals = sorted(set(float(r) for r in rs if r > 0))
        if len(vals) < 2:
            continue
        tol = (vals[0] * vals[1]) ** 0.5
        expect = next(t for t, r in enumerate(rs) if float(r) < tol) + 1
        res = oracle.mapi(A, w0, 5, tol=tol)
        assert res.converged and res.iters == expect, (n, tol, rs)
        done += 1
    assert done >= 10


def test_residual_pin_has_power_against_l2_and_max_norm():
    # the same exact iterates with the residual measured in the l2 or max norm differ from
    # the l1 residual by far more than the tolerance of the pin above
    differ_l2 = differ_max = 0
    for n, A, w0 in cases():
        ws, nus, rs = power_exact(lambda w: mavp_exact(to_fr(A), w), to_fr(w0), 5)
        prev = to_fr(w0)
        for t, w in enumerate(ws):
            d = [float(a - b) for a, b in zip(w, prev)]
            if abs(float(np.sqrt(np.sum(np.square(d)))) - float(rs[t])) > 1e3 * REL:
                differ_l2 += 1
            if abs(max(abs(x) for x in d) - float(rs[t])) > 1e3 * REL:
                differ_max += 1
            prev = w
    assert differ_l2 >= 40 and differ_max >= 40


def test_normaliser_pin_has_power_against_a_signed_sum():
    caught = 0
    for n, A, w0 in cases():
        y = mavp_exact(to_fr(A), to_fr(w0))
        if sum(y, Fr(0)) != sum((abs(v) for v in y), Fr(0)):
            caught += 1
    assert caught >= N_CASES // 3


def test_mapi_min2_and_diamond_are_exact():
    def diamond_exact(a, b):      # eq. (7): sign(a) b + a sign(b)
        return sgn(a) * b + a * sgn(b)

    for op, term in (("min2", min2_exact), ("diamond", diamond_exact)):
        for n, A, w0 in cases()[:16]:
            ws, nus, rs = power_exact(lambda w: mavp_exact(to_fr(A), w, term), to_fr(w0), 4)
            if len(ws) < 4:
                continue
            res = oracle.mapi(A, w0, 4, op=op)
            for t in range(4):
                assert close(res.norms[t], nus[t], float(nus[t])), (op, n, t)
                assert close(res.residuals[t], rs[t], 1.0), (op, n, t)
            for v, e in zip(res.w, ws[-1]):
                assert close(v, e, 1.0), (op, n)


def test_mapi_zero_normaliser_is_degenerate_at_the_exact_step():
    # A (+) w0 = 0 exactly: w0 orthogonal in the min1 sense to every row
    A = np.array([[1.0, 1.0], [0.5, 0.5]])
    w0 = np.array([0.25, -0.25])
    assert mavp_exact(to_fr(A), to_fr(w0)) == [0, 0]
    with pytest.raises(oracle.OracleDegenerate):
        oracle.mapi(A, w0, 3)


# ---------------------------------------------------------------- l1 power iteration (PageRank form)
def test_rpi_l1_iterates_are_exact():
    for n, A, w0 in cases()[:24]:
        ws, nus, rs = power_exact(lambda w: matvec_exact(to_fr(A), w), to_fr(w0), 5)
        if len(ws) < 5:
            continue
        res = oracle.rpi(A, w0, 5, norm="l1")
        for t in range(5):
            assert close(res.norms[t], nus[t], float(nus[t])), (n, t)
            assert close(res.residuals[t], rs[t], 1.0), (n, t)
        for v, e in zip(res.w, ws[-1]):
            assert close(v, e, 1.0)


def test_pagerank_dense_and_split_sums_are_exact_on_tiny_graphs():
    # eq. (11) on graphs of 3..8 nodes with a dangling node: G = alpha H~ + (1 - alpha)/n with
    # the dangling column of H~ equal to 1/n, alpha = 3/4; the exact MAPI iteration on the
    # dense G against both oracle forms
    rng = np.random.default_rng(77)
    alpha = 0.75
    for n in range(3, 9):
        links = {(int(rng.integers(0, n - 1)), int(rng.integers(0, n - 1))) for _ in range(2 * n)}
        links = {(j, i) for j, i in links if j != i}          # source j -> destination i; node n-1 dangling
        outdeg = np.bincount([j for j, _ in links], minlength=n)
        rows = [[] for _ in range(n)]
        for j, i in sorted(links):
            rows[i].append(j)
        row_ptr = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
        col = np.array([j for r in rows for j in r], dtype=np.int32)
        val = np.array([1.0 / outdeg[j] for r in rows for j in r], dtype=np.float32)
        dang = outdeg == 0
        a = Fr(3, 4)
        G = [[(1 - a) / n for _ in range(n)] for _ in range(n)]
        for i in range(n):
            for p in range(row_ptr[i], row_ptr[i + 1]):
                G[i][col[p]] += a * Fr(float(val[p]))
        for j in range(n):
            if dang[j]:
                for i in range(n):
                    G[i][j] = a / n + (1 - a) / n
        w0 = [Fr(1, n)] * n
        ws, nus, rs = power_exact(lambda w: mavp_exact(G, w), w0, 4)
        for form in ("dense", "csr"):
            res = oracle.pagerank(n, row_ptr, col, val, alpha, "mapi", np.full(n, 1.0 / n), 4, form=form)
            for t in range(4):
                assert close(res.norms[t], nus[t], float(nus[t])), (n, form, t)
                assert close(res.residuals[t], rs[t], 1.0), (n, form, t)
            for v, e in zip(res.w, ws[-1]):
                assert close(v, e, 1.0), (n, form)
