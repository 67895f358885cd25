"""PageRank forms of MAPI and RPI on G = alpha H + (1 - alpha)/N 1, eq. (11) (Sec. 3.3).

Test infrastructure only (see the package docstring).

H is given in CSR by destination row: row i lists the sources j of the links
j -> i with value H_ij (column-stochastic).  A node with no out-link (a column of
H that is all zero) is dangling; its column of H is taken as 1/N, so its column
of G is 1/N.  The product is applied to the dense G, as the paper applies power
iteration "to the matrix G".

Pins (tests/test_oracle_pagerank.py):
  * dense_G + the MAPI/RPI loops: RPI with the l1 normaliser reaches the solution
    of the linear system (I - alpha H~) x = (1 - alpha)/N 1 from scipy.linalg.solve.
  * pagerank_mavp_csr: equals the dense product G (+) w (brute force on 2^12
    nodes), for signed and for positive w.
Parity unpinned: the MAPI PageRank fixed point (no closed form).
"""
from __future__ import annotations

import numpy as np

from .core import F64, _power_loop, mavp, term_min1


def dangling_mask(n, col):
    """Boolean mask of nodes with no out-link: node j never appears as a source."""
    return np.bincount(np.asarray(col, dtype=np.int64), minlength=n) == 0


def dense_G(n, row_ptr, col, val, alpha):
    """Dense G of eq. (11) with the dangling columns of H replaced by 1/N."""
    H = np.zeros((n, n), dtype=F64)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    for i in range(n):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            H[i, col[p]] = val[p]
    H[:, dangling_mask(n, col)] = 1.0 / n
    return alpha * H + (1.0 - alpha) / n


def pagerank_mavp_dense(G, w):
    """G (+) w for the dense G (brute force from eq. 11)."""
    return mavp(G, w, "min1")


def _edge_rows(n, row_ptr):
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(row_ptr, dtype=np.int64)))


def pagerank_mavp_csr(n, row_ptr, col, val, alpha, w, dangling=None):
    """G (+) w in O(nnz + N) without forming G.

    Row i of G holds c = (1 - alpha)/N in every column, except 1/N in the dangling
    columns and alpha H_ij + c in the columns of i's in-links.  Splitting the sum
    over j into those three groups:
        y_i = T + Dg + sum_{j in in(i)} [ t(alpha H_ij + c, w_j) - t(c, w_j) ]
        T   = sum_j t(c, w_j),   Dg = sum_{j dangling} [ t(1/N, w_j) - t(c, w_j) ]
    with t the min1 term of eq. (3).  A dangling node has no out-link, so it is
    never an in-link and the groups do not overlap.
    """
    w = np.asarray(w, dtype=F64)
    col = np.asarray(col, dtype=np.int64)
    if dangling is None:
        dangling = dangling_mask(n, col)
    c = (1.0 - alpha) / n
    T = np.sum(term_min1(c, w))
    Dg = np.sum(term_min1(1.0 / n, w[dangling]) - term_min1(c, w[dangling]))
    g = alpha * np.asarray(val, dtype=F64) + c
    wj = w[col]
    edge = term_min1(g, wj) - term_min1(c, wj)
    y = np.bincount(_edge_rows(n, row_ptr), weights=edge, minlength=n)
    return T + Dg + y


def pagerank_rpi_csr(n, row_ptr, col, val, alpha, w, dangling=None):
    """G w without forming G: alpha H w + alpha/N sum_{j dangling} w_j + (1-alpha)/N sum_j w_j."""
    w = np.asarray(w, dtype=F64)
    col = np.asarray(col, dtype=np.int64)
    if dangling is None:
        dangling = dangling_mask(n, col)
    hw = np.bincount(_edge_rows(n, row_ptr), weights=np.asarray(val, dtype=F64) * w[col], minlength=n)
    return alpha * hw + alpha / n * np.sum(w[dangling]) + (1.0 - alpha) / n * np.sum(w)


def pagerank(n, row_ptr, col, val, alpha, method, w0, T, tol=0.0, form="csr"):
    """Power iteration on G (eq. 11) with the l1 normaliser, for MAPI (eq. 6) or RPI (eq. 1).

    ``form`` "dense" builds G explicitly (small n only); "csr" uses the split sums.
    """
    dangling = dangling_mask(n, col)
    if form == "dense":
        G = dense_G(n, row_ptr, col, val, alpha)
        if method == "mapi":
            step = lambda w: mavp(G, w, "min1")  # noqa: E731
        else:
            step = lambda w: G @ w  # noqa: E731
    else:
        if method == "mapi":
            step = lambda w: pagerank_mavp_csr(n, row_ptr, col, val, alpha, w, dangling)  # noqa: E731
        else:
            step = lambda w: pagerank_rpi_csr(n, row_ptr, col, val, alpha, w, dangling)  # noqa: E731
    return _power_loop(step, w0, T, tol, "l1")
