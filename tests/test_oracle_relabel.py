"""Pins of oracle.relabel (degree-ordered labelling, Sec. 5.3.1 / Table 6) against
what the definition fixes: a hand-worked example, bijection and order
invariants, isomorphism of the edge sets, PageRank equivariance (through the
independent C PageRank of the oracle), a star graph, and a planted mistake."""
import numpy as np
import pytest

import graphgen
import oracle


def _edges(row_off, col):
    row_off = np.asarray(row_off)
    src = np.repeat(np.arange(len(row_off) - 1), np.diff(row_off))
    return src, np.asarray(col)


def test_hand_worked_example():
    # edges 0->1, 0->2, 1->2, 3->0, 3->2; in-degrees 1, 1, 3, 0:
    # node 2 gets label 0, then nodes 0, 1 (equal in-degree, old ID order), then 3.
    # New edges: 1->2, 1->0, 2->0, 3->1, 3->0 -> rows [], [0, 2], [0], [0, 1].
    perm, ro, c = oracle.relabel([0, 2, 3, 3, 5], [1, 2, 2, 0, 2], key="in")
    assert perm.tolist() == [1, 2, 0, 3]
    assert ro.tolist() == [0, 0, 2, 3, 5]
    assert c.tolist() == [0, 2, 0, 0, 1]
    # by out-degree (2, 1, 0, 2): nodes 0, 3, then 1, then 2
    perm, ro, c = oracle.relabel([0, 2, 3, 3, 5], [1, 2, 2, 0, 2], key="out")
    assert perm.tolist() == [0, 2, 3, 1]
    # new edges 0->2, 0->3, 2->3, 1->0, 1->3
    assert ro.tolist() == [0, 2, 4, 5, 5]
    assert c.tolist() == [2, 3, 0, 3, 3]


def _check_invariants(row_off, col, key):
    n = len(row_off) - 1
    perm, ro2, c2 = oracle.relabel(row_off, col, key=key)
    assert np.array_equal(np.sort(perm), np.arange(n))  # bijection
    deg = np.bincount(col, minlength=n) if key == "in" else np.diff(row_off)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    d_new = deg[inv]
    assert np.all(np.diff(d_new) <= 0)  # largest degree first
    ties = np.diff(d_new) == 0
    assert np.all(np.diff(inv)[ties] > 0)  # equal degrees keep old-ID order
    # the relabelled degrees are the old ones moved
    d2 = np.bincount(c2, minlength=n) if key == "in" else np.diff(ro2)
    assert np.array_equal(d2, d_new)
    # same edge set under perm; rows strictly ascending
    s, d = _edges(row_off, col)
    s2, dd2 = _edges(ro2, c2)
    a = np.sort(perm[s] * n + perm[d])
    b = s2 * n + dd2
    assert np.array_equal(a, b)
    assert np.all(np.diff(b) > 0)
    return perm, ro2, c2


@pytest.mark.parametrize("key", ["in", "out"])
@pytest.mark.parametrize("seed", [1, 2])
def test_invariants_rmat(key, seed):
    r, c = graphgen.rmat(12, 8, seed=seed, relabel="random")
    _check_invariants(r, c, key)


@pytest.mark.parametrize("key", ["in", "out"])
def test_pagerank_equivariant(key):
    r, c = graphgen.rmat(11, 16, seed=3, relabel="random")
    perm, ro2, c2 = _check_invariants(r, c, key)
    a = oracle.pagerank(r, c, d=0.85, iters=30).x
    b = oracle.pagerank(ro2, c2, d=0.85, iters=30).x
    np.testing.assert_allclose(b[perm], a, rtol=1e-12, atol=1e-15)


def test_star_and_degenerate():
    n = 9  # every leaf points at node 5
    leaves = [u for u in range(n) if u != 5]
    edges = np.array([[u, 5] for u in leaves])
    r, c = graphgen.from_edges(n, edges[:, 0], edges[:, 1], threads=1)
    perm, ro2, c2 = oracle.relabel(r, c, key="in")
    assert perm[5] == 0 and perm[leaves].tolist() == list(range(1, n))
    assert np.all(c2 == 0)
    perm, ro2, c2 = oracle.relabel(r, c, key="out")
    assert perm[5] == n - 1  # the only node without out-edges goes last
    # no edges: identity
    perm, ro2, c2 = oracle.relabel(np.zeros(5, np.int64), np.zeros(0, np.int64))
    assert perm.tolist() == [0, 1, 2, 3] and len(c2) == 0


def test_planted_tie_order_mistake_is_caught():
    r, c = graphgen.rmat(10, 8, seed=5, relabel="random")
    n = len(r) - 1
    deg = np.bincount(c, minlength=n)
    bad = np.lexsort((-np.arange(n), -deg))  # ties in decreasing old ID
    perm_bad = np.empty(n, np.int64)
    perm_bad[bad] = np.arange(n)
    perm, _, _ = oracle.relabel(r, c, key="in")
    assert not np.array_equal(perm, perm_bad)
    inv = np.empty(n, np.int64)
    inv[perm_bad] = np.arange(n)
    ties = np.diff(deg[inv]) == 0
    assert not np.all(np.diff(inv)[ties] > 0)
