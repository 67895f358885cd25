"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This module holds no arithmetic of the method (no vector product, no iteration,
no normalisation of iterates): it only draws matrices, start vectors and graphs
from a seed, in the shapes and distributions of the paper's workloads.  Both the
oracle and the HIP library receive the same bytes from here.

Host draws use numpy's PCG64 (``numpy.random.default_rng(seed)``) in the draw
order written in each docstring.  The large dense covariance can instead be
drawn on a torch device (``device="cuda"``) with torch's seeded generator; the
two sources give different, equally valid, matrices for one seed.
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.default_rng(int(seed))


# --------------------------------------------------------------------------
# Dense symmetric covariance inputs
# --------------------------------------------------------------------------
def dense_cov(n, N, seed, device=None):
    """C = X X^T / N as float32, X of shape n x N with i.i.d. N(0,1) entries, rows centred.

    Draw order (host): X = rng.standard_normal((n, N)).  The product is formed in
    float64 and rounded once to float32.  With ``device`` set, X is drawn by
    torch.randn on that device from torch.Generator(device).manual_seed(seed) and
    the float64 product is formed there; a torch tensor is returned.
    """
    if device is None:
        X = _rng(seed).standard_normal((n, N))
        X -= X.mean(axis=1, keepdims=True)
        return ((X @ X.T) / N).astype(np.float32)
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    X = torch.randn((n, N), generator=g, device=device, dtype=torch.float32).double()
    X -= X.mean(dim=1, keepdim=True)
    C = (X @ X.T) / N
    del X
    out = C.float().contiguous()
    del C
    return out


def start_vector(n, seed):
    """b0 ~ U(-1, 1)^n scaled to unit l2 norm (Algorithm 1 starts from ||w0|| = 1), float32."""
    b = _rng(seed).uniform(-1.0, 1.0, size=n)
    b /= np.sqrt(np.sum(b * b))
    return b.astype(np.float32)


def start_vectors(n, k, seed):
    """k start vectors as the columns of an n x k float32 array (column i from seed + i)."""
    return np.stack([start_vector(n, seed + i) for i in range(k)], axis=1)


def uniform_start(n):
    """The uniform PageRank start vector 1/n (float32)."""
    return np.full(n, 1.0 / n, dtype=np.float32)


def dyadic_matrix(n_rows, n_cols, seed, denom_pow=3, max_num=16):
    """Entries k / 2^denom_pow with integer k uniform in [-max_num, max_num].

    Such values keep every sign, min and partial sum of a few thousand terms exact
    in float32, so a product over them has one correct float32 answer.
    """
    k = _rng(seed).integers(-max_num, max_num + 1, size=(n_rows, n_cols))
    return (k / float(2 ** denom_pow)).astype(np.float32)


def dyadic_vector(n, seed, denom_pow=3, max_num=16):
    return dyadic_matrix(1, n, seed, denom_pow, max_num)[0]


def planted_symmetric(n, gaps, seed):
    """Q diag(lam) Q^T (float32) with a random orthogonal Q and eigenvalues
    lam = [1, 1-g1, 1-g1-g2, ...] followed by a bulk uniform in [0, lam_last/2].

    Draw order: G = rng.standard_normal((n, n)); Q from numpy's QR of G;
    bulk = rng.uniform(size=n - len(gaps) - 1).
    """
    rng = _rng(seed)
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))[None, :]
    lam = [1.0]
    for g in gaps:
        lam.append(lam[-1] - g)
    bulk = rng.uniform(size=n - len(lam)) * lam[-1] * 0.5
    d = np.concatenate([np.array(lam), np.sort(bulk)[::-1]])
    return ((Q * d[None, :]) @ Q.T).astype(np.float32), Q, d


# --------------------------------------------------------------------------
# PCA data matrix (low-rank factors + noise + Laplace outliers)
# --------------------------------------------------------------------------
def pca_data(D, N, seed, n_factors=16, noise=0.1, outlier_frac=0.05, laplace_b=10.0,
             decay=0.8, lead=2.0):
    """X of shape D x N (columns are samples), float32, rows zero-meaned.

    x_k = sum_f u_f z_fk + noise * e_k with u_f ~ N(0, I_D) and
    z_fk ~ N(0, (lead * decay^(f-1))^2); then a fraction ``outlier_frac`` of the
    entries is replaced by Laplace(0, laplace_b) draws; then every row is centred.
    Draw order: U (D x F), Z (F x N), E (D x N), outlier mask (D x N uniform),
    Laplace values (one per masked entry).
    """
    rng = _rng(seed)
    U = rng.standard_normal((D, n_factors))
    sd = lead * decay ** np.arange(n_factors)
    Z = rng.standard_normal((n_factors, N)) * sd[:, None]
    X = U @ Z
    X += noise * rng.standard_normal((D, N))
    mask = rng.uniform(size=(D, N)) < outlier_frac
    X[mask] = rng.laplace(0.0, laplace_b, size=int(mask.sum()))
    X -= X.mean(axis=1, keepdims=True)
    return X.astype(np.float32)


def laplace_from_uniform(r, b):
    """Laplace(0, b) draws from uniforms r in [0, 1) (torch tensor) by the inverse CDF
    x = -b sign(u) log(1 - 2|u|), u = r - 1/2.  |u| is clamped to 1/2 - 2^-25 so that
    r = 0, which float32 uniform generators do return, gives -b log(2^-24) instead of an
    infinity; every draw is finite, |x| <= 24 b log 2."""
    import torch
    u = r - 0.5
    a = torch.clamp(torch.abs(u), max=0.5 - 2.0 ** -25)
    return -b * torch.sign(u) * torch.log1p(-2.0 * a)


def pca_data_device(D, N, seed, device, n_factors=16, noise=0.1, outlier_frac=0.05, laplace_b=10.0,
                    decay=0.8, lead=2.0):
    """``pca_data`` drawn with torch's seeded generator on ``device``; returns (X, X_clean)
    as float32 tensors (X_clean: the centred low-rank part U Z).  Same recipe and draw
    order as ``pca_data``; the Laplace draws are inverse-CDF transforms of uniforms
    (``laplace_from_uniform``)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    U = torch.randn((D, n_factors), generator=g, device=device, dtype=torch.float32)
    sd = lead * decay ** torch.arange(n_factors, device=device, dtype=torch.float32)
    Z = torch.randn((n_factors, N), generator=g, device=device, dtype=torch.float32) * sd[:, None]
    clean = U @ Z
    X = clean + noise * torch.randn((D, N), generator=g, device=device, dtype=torch.float32)
    mask = torch.rand((D, N), generator=g, device=device) < outlier_frac
    r = torch.rand((D, N), generator=g, device=device, dtype=torch.float32)
    X = torch.where(mask, laplace_from_uniform(r, laplace_b), X)
    X -= X.mean(dim=1, keepdim=True)
    clean -= clean.mean(dim=1, keepdim=True)
    return X.contiguous(), clean.contiguous()


def pca_clean(D, N, seed, n_factors=16, decay=0.8, lead=2.0):
    """The noise- and outlier-free low-rank part U Z of ``pca_data`` for the same seed,
    centred, float64 (for the reconstruction-error report)."""
    rng = _rng(seed)
    U = rng.standard_normal((D, n_factors))
    sd = lead * decay ** np.arange(n_factors)
    Z = rng.standard_normal((n_factors, N)) * sd[:, None]
    X = U @ Z
    X -= X.mean(axis=1, keepdims=True)
    return X


# --------------------------------------------------------------------------
# Power-law directed graphs, CSR by destination row
# --------------------------------------------------------------------------
def powerlaw_graph(n, seed, avg_deg=16.0, zipf_a=2.1, dangling_frac=0.05):
    """Directed graph with Zipf out-degrees and uniform destinations, as column-stochastic CSR.

    Draw order: z = rng.zipf(zipf_a, n); out-degree d_i = min(n-1, floor(z_i *
    avg_deg / mean(z))); a set of round(dangling_frac * n) nodes drawn by
    rng.choice(n, size, replace=False) gets d_i = 0; then, for all edges at once,
    u = rng.integers(0, n-1, sum(d)) and destination = u + (u >= source) (uniform
    over the other nodes).  Repeated (source, destination) pairs are merged.
    Value H_ij = 1 / (distinct out-degree of j), rounded to float32.

    Returns dict(n, row_ptr int32[n+1], col int32[nnz] (sources), val float32[nnz],
    outdeg int32[n]); rows are destinations, columns within a row ascend.
    """
    rng = _rng(seed)
    z = rng.zipf(zipf_a, n).astype(np.float64)
    d = np.minimum(n - 1, np.floor(z * avg_deg / z.mean())).astype(np.int64)
    n_dang = int(round(dangling_frac * n))
    if n_dang:
        d[rng.choice(n, size=n_dang, replace=False)] = 0
    src = np.repeat(np.arange(n, dtype=np.int64), d)
    u = rng.integers(0, n - 1, size=src.shape[0], dtype=np.int64) if n > 1 else np.zeros(0, np.int64)
    dst = u + (u >= src)
    key = np.unique(dst * n + src)
    dst = key // n
    src = key % n
    outdeg = np.bincount(src, minlength=n)
    val = (1.0 / outdeg[src]).astype(np.float32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(dst, minlength=n), out=row_ptr[1:])
    return dict(n=n, row_ptr=row_ptr.astype(np.int32), col=src.astype(np.int32),
                val=val, outdeg=outdeg.astype(np.int32))


def tiny_graph(edges, n):
    """Column-stochastic CSR (by destination) of an explicit edge list [(src, dst), ...]."""
    src = np.array([e[0] for e in edges], dtype=np.int64)
    dst = np.array([e[1] for e in edges], dtype=np.int64)
    key = np.unique(dst * n + src)
    dst, src = key // n, key % n
    outdeg = np.bincount(src, minlength=n)
    val = (1.0 / outdeg[src]).astype(np.float32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(dst, minlength=n), out=row_ptr[1:])
    return dict(n=n, row_ptr=row_ptr.astype(np.int32), col=src.astype(np.int32),
                val=val, outdeg=outdeg.astype(np.int32))


# --------------------------------------------------------------------------
# Counter-based generated problems (the device generator's definition)
# --------------------------------------------------------------------------
_U64 = np.uint64


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea and Flood, 2014) on uint64 arrays, mod 2^64."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = x + _U64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> _U64(27))) * _U64(0x94D049BB133111EB)
    return x ^ (x >> _U64(31))


def _counter(base, k):
    with np.errstate(over="ignore"):
        return splitmix64(base + np.asarray(k, dtype=np.uint64))


def generated_dense(n, seed):
    """The seed-generated symmetric problem: (A float32 n x n, w0 float32 n).

    a_ij = fl32(fl32(x_ij * s_n) + sigma_i sigma_j * fl32(6 / n)), x_ij = (top 24 bits of
    splitmix64(splitmix64(seed) + (min(i,j) << 32 | max(i,j)))) - 2^23, s_n = fl32(sqrt(3) /
    (2^23 sqrt(n))), sigma_i = -1 if the top bit of splitmix64(splitmix64(seed ^ 0x5BD1E995) + i)
    is set else +1.  w0_i = -+fl32(1 / sqrt(n)) by the top bit of
    splitmix64(splitmix64(seed ^ 0x1B873593) + i).
    """
    seed = _U64(seed)
    base = splitmix64(seed)
    sbase = splitmix64(seed ^ _U64(0x5BD1E995))
    idx = np.arange(n, dtype=np.uint64)
    lo = np.minimum(idx[:, None], idx[None, :])
    hi = np.maximum(idx[:, None], idx[None, :])
    h = _counter(base, (lo << _U64(32)) | hi)
    x = ((h >> _U64(40)).astype(np.int64) - 8388608).astype(np.float32)
    s_n = np.float32(1.7320508075688772 / (8388608.0 * np.sqrt(float(n))))
    spike = np.float32(6.0 / float(n))
    sig = (_counter(sbase, idx) >> _U64(63)).astype(bool)
    same = sig[:, None] == sig[None, :]
    A = (x * s_n).astype(np.float32) + np.where(same, spike, -spike).astype(np.float32)
    return A.astype(np.float32), generated_start(n, seed)


def generated_start(n, seed):
    """The start vector of the seed-generated problem (generated_dense) alone: w0_i =
    -+fl32(1 / sqrt(n)) by the top bit of splitmix64(splitmix64(seed ^ 0x1B873593) + i)."""
    vbase = splitmix64(_U64(seed) ^ _U64(0x1B873593))
    idx = np.arange(n, dtype=np.uint64)
    inv = np.float32(1.0 / np.sqrt(float(n)))
    return np.where((_counter(vbase, idx) >> _U64(63)).astype(bool), -inv, inv).astype(np.float32)


# --------------------------------------------------------------------------
# Sec. 3.2 construction (stochastic PCA comparison) and mini-batch indices
# --------------------------------------------------------------------------
def sec32_data(N, D, seed, gap=0.1):
    """X = sqrt(N) U Sigma V^T of shape N x D (samples as rows), float32, with U (N x D) and V
    (D x D) having orthonormal columns and Sigma = diag(1, sqrt(1-gap), ..., sqrt(1-gap)), so
    that the covariance X^T X / N of eq. (2) is V diag(1, 1-gap, ...) V^T, with eigen-gap `gap`
    and top eigenvector V[:, 0] (Sec. 3.2: N = 10^6, D = 10, gap 0.1).  The sqrt(N) puts the
    samples on a unit scale (entries ~ 1), comparable to an l1-normalised iterate in D = 10:
    the operator of eq. (3) is only jointly homogeneous, and with entries ~ 1e-3 the product
    would see only the signs of w.  Returns (X, v1) with v1 float64.

    Draw order: G = rng.standard_normal((N, D)); U from numpy's QR of G (signs fixed by
    diag R); H = rng.standard_normal((D, D)); V from the QR of H likewise.
    """
    rng = _rng(seed)
    G = rng.standard_normal((N, D))
    U, R = np.linalg.qr(G)
    U = U * np.sign(np.diag(R))[None, :]
    H = rng.standard_normal((D, D))
    V, R2 = np.linalg.qr(H)
    V = V * np.sign(np.diag(R2))[None, :]
    sig = np.full(D, np.sqrt(1.0 - gap))
    sig[0] = 1.0
    X = np.sqrt(N) * ((U * sig[None, :]) @ V.T)
    return X.astype(np.float32), V[:, 0].copy()


def minibatch_indices(runs, T, s, N, seed):
    """I.i.d. uniform sample indices in [0, N) for Algorithm 3's mini batches, int32 of shape
    (runs, T, s): rng.integers(0, N, size=(runs, T, s))."""
    return _rng(seed).integers(0, N, size=(runs, T, s)).astype(np.int32)


# --------------------------------------------------------------------------
# Occluded images (Sec. 3.1 structure, synthetic content)
# --------------------------------------------------------------------------
def occluded_images(D, N, seed, tiles=4, bad_tiles=3):
    """A synthetic D x D gray-scale image in [0, 1] and N corrupted copies (Sec. 3.1: the image
    is cut into tiles x tiles tiles and, in each copy, `bad_tiles` tiles drawn at random are
    replaced by i.i.d. U[0, 1] noise).  The paper's images are not available; the clean image is
    a smooth pattern: 0.5 + 0.25 sin(2 pi u f1) cos(2 pi v f2) plus three Gaussian blobs, clipped
    to [0, 1].  Returns (clean float32 (D*D,), V float32 (D*D, N)) with pixels in row-major order.

    Draw order: f1, f2 = rng.uniform(1, 3, 2); blob centres rng.uniform(0, 1, (3, 2)), widths
    rng.uniform(0.05, 0.2, 3), heights rng.uniform(-0.4, 0.4, 3); then per copy
    rng.choice(tiles * tiles, bad_tiles, replace=False) and the noise of those tiles in order.
    """
    rng = _rng(seed)
    u, v = np.meshgrid(np.linspace(0.0, 1.0, D), np.linspace(0.0, 1.0, D), indexing="ij")
    f1, f2 = rng.uniform(1.0, 3.0, 2)
    img = 0.5 + 0.25 * np.sin(2 * np.pi * u * f1) * np.cos(2 * np.pi * v * f2)
    cen = rng.uniform(0.0, 1.0, (3, 2))
    wid = rng.uniform(0.05, 0.2, 3)
    hgt = rng.uniform(-0.4, 0.4, 3)
    for b in range(3):
        img += hgt[b] * np.exp(-((u - cen[b, 0]) ** 2 + (v - cen[b, 1]) ** 2) / (2 * wid[b] ** 2))
    img = np.clip(img, 0.0, 1.0)
    t = D // tiles
    V = np.empty((D * D, N), dtype=np.float32)
    for i in range(N):
        x = img.copy()
        for tt in rng.choice(tiles * tiles, bad_tiles, replace=False):
            r, c = divmod(int(tt), tiles)
            x[r * t:(r + 1) * t, c * t:(c + 1) * t] = rng.uniform(0.0, 1.0, (t, t))
        V[:, i] = x.reshape(-1)
    return img.reshape(-1).astype(np.float32), V
