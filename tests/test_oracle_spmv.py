"""Pins of the oracle's SpMV (Sec. 3.5): independent computations of the
same product, closed forms, and the bin order of the weights against the
C oracle's PNG layout."""
import numpy as np
import pytest

import graphgen
import oracle


def dense(row_off, col, weights=None):
    n = len(row_off) - 1
    A = np.zeros((n, n))
    for u in range(n):
        for e in range(row_off[u], row_off[u + 1]):
            A[u, col[e]] += 1.0 if weights is None else float(weights[e])
    return A


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spmv_equals_dense_transpose_product(seed):
    rng = np.random.default_rng(seed)
    r, c = graphgen.rmat(6, 5, seed=seed, relabel="random")
    w = rng.standard_normal(len(c))
    x = rng.standard_normal(len(r) - 1)
    np.testing.assert_allclose(oracle.spmv(r, c, x, w), dense(r, c, w).T @ x, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.spmv(r, c, x), dense(r, c).T @ x, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("rows,cols", [(7, 19), (23, 5), (9, 9)])
def test_rectangular_spmv_with_diagonal_equals_dense_product(rows, cols):
    """A non-square matrix with diagonal entries (Sec. 3.5): y has one entry
    per column, y = A^T x by the dense product."""
    rng = np.random.default_rng(rows * 31 + cols)
    A = np.where(rng.random((rows, cols)) < 0.35, rng.standard_normal((rows, cols)), 0.0)
    for i in range(min(rows, cols)):
        A[i, i] = float(i + 1)  # every diagonal entry present
    u, v = np.nonzero(A)
    r = np.zeros(rows + 1, np.int32)
    r[1:] = np.cumsum(np.bincount(u, minlength=rows))
    w = A[u, v]
    x = rng.standard_normal(rows)
    y = oracle.spmv(r, v, x, w, num_cols=cols)
    assert y.shape == (cols,)
    np.testing.assert_allclose(y, A.T @ x, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.spmv(r, v, x, num_cols=cols), (A != 0).T @ x, rtol=1e-12, atol=1e-12)


def test_spmv_star_and_cycle():
    n = 6
    # in-star: every leaf points at node 0
    r, c = graphgen.from_edges(n, np.arange(1, n), np.zeros(n - 1, np.int32))
    x = np.arange(n, dtype=np.float64) + 1.0
    y = oracle.spmv(r, c, x)
    assert y[0] == x[1:].sum() and np.all(y[1:] == 0.0)
    # weighted cycle u -> u+1: y(v) = w(v-1, v) x(v-1)
    src = np.arange(n)
    dst = (src + 1) % n
    r, c = graphgen.from_edges(n, src, dst)
    w = np.array([2.0, -3.0, 0.5, 7.0, -1.0, 4.0])  # weights in CSR order = by source here
    y = oracle.spmv(r, c, x, w)
    np.testing.assert_array_equal(y, np.roll(w * x, 1))


def test_spmv_with_inverse_out_degrees_is_a_pagerank_step():
    """PageRank's push-pull sum is the SpMV with w(u,v) = 1/outdeg(u); one step
    of Eq. 1 adds the jump and the dangling share (two different oracle
    routes: numpy push here, C pull in step_at)."""
    r, c = graphgen.rmat(10, 8, seed=5, relabel="random")
    n = len(r) - 1
    outdeg = np.diff(r)
    w = 1.0 / np.repeat(outdeg, outdeg)
    x = np.random.default_rng(1).random(n)
    d = 0.85
    dang = x[outdeg == 0].sum()
    y = d * oracle.spmv(r, c, x, w) + (1 - d) / n + d * dang / n
    nodes = np.arange(n)
    np.testing.assert_allclose(y, oracle.step_at(r, c, x, nodes, d=d), rtol=1e-12, atol=1e-15)


def test_spmv_is_linear():
    rng = np.random.default_rng(3)
    r, c = graphgen.rmat(9, 6, seed=2)
    w = rng.standard_normal(len(c))
    a, b = rng.standard_normal(len(r) - 1), rng.standard_normal(len(r) - 1)
    np.testing.assert_allclose(oracle.spmv(r, c, 2.5 * a - b, w), 2.5 * oracle.spmv(r, c, a, w) - oracle.spmv(r, c, b, w),
                               rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("q", [1, 3, 8, 64])
def test_bin_weights_follow_the_destination_id_order(q):
    """Weights that encode their own edge (w = destination ID) come out in the
    order of the C oracle's destination-ID bins; a wrong key order (inside a
    bin by destination, then source) does not."""
    r, c = graphgen.rmat(8, 6, seed=q, relabel="random")
    png = oracle.png_layout(r, c, q)
    ids = (png.did & 0x7FFFFFFF).astype(np.int64)
    wb = oracle.bin_weights(r, c, c.astype(np.float64), q)
    np.testing.assert_array_equal(wb, ids)
    # and a weight naming the source: the bins are ordered by source partition, then source
    src = np.repeat(np.arange(len(r) - 1), np.diff(r))
    ws = oracle.bin_weights(r, c, src.astype(np.float64), q)
    for p in range(png.k):
        seg = ws[png.did_start[p]:png.did_start[p + 1]]
        assert np.all(np.diff(seg) >= 0)
    if q > 1:  # with q = 1 a bin holds one destination and the two orders coincide
        wrong = np.asarray(c)[np.lexsort((src, c, np.asarray(c) // q))]
        assert not np.array_equal(wrong, ids)
