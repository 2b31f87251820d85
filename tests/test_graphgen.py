"""The seeded input generator: determinism, canonical form, configured sizes."""
import numpy as np
import pytest

import graphgen


def _canonical(r, c):
    n = len(r) - 1
    assert r[0] == 0 and r[-1] == len(c) and np.all(np.diff(r) >= 0)
    assert np.all((c >= 0) & (c < n))
    src = np.repeat(np.arange(n), np.diff(r))
    assert not np.any(src == c)  # no self-loops
    # strictly ascending inside each row <=> sorted and no duplicates
    same_row = src[1:] == src[:-1]
    assert np.all(c[1:][same_row] > c[:-1][same_row])


@pytest.mark.parametrize("relabel", [None, "random", "indegree"])
def test_rmat_canonical_and_deterministic(relabel):
    a = graphgen.rmat(12, 16, seed=3, relabel=relabel, threads=1)
    b = graphgen.rmat(12, 16, seed=3, relabel=relabel, threads=4)
    _canonical(*a)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    c = graphgen.rmat(12, 16, seed=4, relabel=relabel)
    assert not np.array_equal(a[1][: len(c[1])], c[1][: len(a[1])])


def test_relabels_are_isomorphic():
    r, c = graphgen.rmat(11, 8, seed=5)
    rr, cr = graphgen.rmat(11, 8, seed=5, relabel="random")
    ri, ci = graphgen.rmat(11, 8, seed=5, relabel="indegree")
    assert len(c) == len(cr) == len(ci)
    assert sorted(np.diff(r)) == sorted(np.diff(rr)) == sorted(np.diff(ri))
    indeg = np.bincount(ci, minlength=len(ri) - 1)
    assert np.all(np.diff(indeg) <= 0)  # in-degree descending


def test_configured_rmat16_size():
    """RMAT scale 16, edge factor 16, (.57,.19,.19,.05): 1,048,576 draws, about
    0.95M edges after dropping self-loops and duplicates."""
    r, c = graphgen.rmat(16, 16, seed=1)
    assert len(r) == 65537
    assert 0.90e6 < len(c) < 1.0e6
    frac_dangling = (np.diff(r) == 0).mean()
    assert 0.3 < frac_dangling < 0.45


def test_uniform_and_edge_lists():
    r, c = graphgen.uniform(1000, 20000, seed=4)
    _canonical(r, c)
    assert 19000 < len(c) <= 20000
    r, c = graphgen.from_edges(4, [0, 0, 0, 1, 3, 2], [1, 1, 0, 2, 0, 2])
    assert r.tolist() == [0, 1, 2, 2, 3] and c.tolist() == [1, 2, 0]


def test_seed_sets():
    off, s = graphgen.seed_sets(1000, 16, seed=3)
    sizes = np.diff(off)
    assert len(sizes) == 16 and sizes.min() >= 1 and sizes.max() <= 100
    for j in range(16):
        g = s[off[j]:off[j + 1]]
        assert len(np.unique(g)) == len(g) and g.min() >= 0 and g.max() < 1000
