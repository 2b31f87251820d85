"""Pins for the CPU oracle: each checks it against something other than itself.

* closed forms and special cases that the recurrence of Eq. 1 (Sec. 2.1) fixes,
* the dense Google-matrix form of Eq. 2 (power iteration and a linear solve),
* the contraction of the recurrence and its a-posteriori error bound,
* the Sec. 3.1 worked example of write offsets (tests/golden),
* a brute-force set construction of the PNG layout (Sec. 3.3),
* the PNG route of Alg. 3 + Alg. 5 reproducing the pull route of Alg. 1.

The closed forms are derived from the fixed-point equation with uniform
dangling redistribution; the derivations are in the docstrings.
"""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr(n, edges):
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return graphgen.from_edges(n, edges[:, 0], edges[:, 1], threads=1)


def random_digraph(n, p, seed, dangling_frac=0.3):
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < p
    np.fill_diagonal(a, False)
    dang = rng.random(n) < dangling_frac
    a[dang, :] = False
    u, v = np.nonzero(a)
    return csr(n, np.stack([u, v], 1))


def dense_google(row_off, col, d, t):
    """G = d (M + t delta^T) + (1-d) t 1^T with M[v,u] = 1/outdeg(u) for u->v
    and delta the indicator of dangling nodes (Eq. 2 plus dangling spread)."""
    n = len(row_off) - 1
    M = np.zeros((n, n))
    delta = np.zeros(n)
    for u in range(n):
        nb = col[row_off[u]:row_off[u + 1]]
        if len(nb) == 0:
            delta[u] = 1.0
        for v in nb:
            M[v, u] += 1.0 / len(nb)
    return d * (M + np.outer(t, delta)) + (1 - d) * np.outer(t, np.ones(n))


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mass_is_conserved_every_iteration(seed):
    r, c = graphgen.rmat(10, 8, seed=seed)
    for it in range(1, 6):
        x = oracle.pagerank(r, c, iters=it).x
        assert abs(x.sum() - 1.0) < 1e-12
        assert np.all(x > 0)


def test_directed_cycle_is_uniform_every_iteration():
    n = 37
    r, c = csr(n, [(i, (i + 1) % n) for i in range(n)])
    for it in (1, 2, 7):
        x = oracle.pagerank(r, c, d=0.85, iters=it).x
        np.testing.assert_allclose(x, 1.0 / n, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [5, 9])
def test_in_star_closed_form(n):
    """Leaves 1..n-1 point at the centre 0, which is dangling.  Fixed point:
    x_l = (1-d)/n + d x_c/n and x_c + (n-1) x_l = 1 give
    x_l = 1/(n+(n-1)d), x_c = (1+(n-1)d)/(n+(n-1)d)."""
    d = 0.85
    r, c = csr(n, [(i, 0) for i in range(1, n)])
    res = oracle.pagerank(r, c, d=d, iters=500, tol=1e-15)
    x = res.x
    xl = 1.0 / (n + (n - 1) * d)
    xc = (1 + (n - 1) * d) / (n + (n - 1) * d)
    bound = d * res.resid / (1 - d) + 1e-15
    assert abs(x[0] - xc) <= bound
    assert np.max(np.abs(x[1:] - xl)) <= bound
    if n == 5:  # the closed form's values at n = 5, d = 0.85
        assert round(xc, 7) == 0.5238095 and round(xl, 7) == 0.1190476


@pytest.mark.parametrize("n", [5, 9])
def test_out_star_closed_form(n):
    """Centre 0 points at n-1 dangling leaves.  x_c = (1-d)/n + d(1-x_c)/n gives
    x_c = 1/(n+d); the leaves share 1-x_c equally."""
    d = 0.85
    r, c = csr(n, [(0, i) for i in range(1, n)])
    res = oracle.pagerank(r, c, d=d, iters=500, tol=1e-15)
    xc = 1.0 / (n + d)
    xl = (n + d - 1) / ((n + d) * (n - 1))
    bound = d * res.resid / (1 - d) + 1e-15
    assert abs(res.x[0] - xc) <= bound
    assert np.max(np.abs(res.x[1:] - xl)) <= bound
    if n == 5:
        assert round(xc, 7) == 0.1709402 and round(xl, 7) == 0.2072650


def test_bidirected_star_closed_form():
    """Centre <-> leaves, no dangling node: x_c = (1-d)/n + d(1-x_c) gives
    x_c = (1+(n-1)d)/(n(1+d))."""
    n, d = 5, 0.85
    e = [(0, i) for i in range(1, n)] + [(i, 0) for i in range(1, n)]
    r, c = csr(n, e)
    res = oracle.pagerank(r, c, d=d, iters=500, tol=1e-15)
    xc = (1 + (n - 1) * d) / (n * (1 + d))
    assert abs(res.x[0] - xc) <= d * res.resid / (1 - d) + 1e-15
    assert round(xc, 7) == 0.4756757


def test_degenerate_graphs_are_uniform():
    n = 11
    # no edges at all: every node dangling, y = (1-d)/n + d/n
    r, c = csr(n, np.zeros((0, 2)))
    np.testing.assert_allclose(oracle.pagerank(r, c, iters=3).x, 1 / n, rtol=1e-15)
    # complete digraph
    e = [(u, v) for u in range(n) for v in range(n) if u != v]
    r, c = csr(n, e)
    np.testing.assert_allclose(oracle.pagerank(r, c, iters=3).x, 1 / n, rtol=1e-14)
    # d = 0: only the jump term survives
    r, c = graphgen.rmat(8, 8, seed=5)
    np.testing.assert_allclose(oracle.pagerank(r, c, d=0.0, iters=1).x, 1 / 256, rtol=1e-15)
    # a single node
    r, c = csr(1, np.zeros((0, 2)))
    assert oracle.pagerank(r, c, iters=4).x[0] == 1.0


# ---------------------------------------------------------- dense brute force

@pytest.mark.parametrize("seed,n,p,d", [(1, 12, 0.3, 0.85), (2, 40, 0.1, 0.85), (3, 64, 0.05, 0.5),
                                        (4, 64, 0.2, 0.99), (5, 7, 0.5, 0.15)])
def test_dense_power_iteration_matches_every_iterate(seed, n, p, d):
    r, c = random_digraph(n, p, seed)
    t = np.full(n, 1.0 / n)
    G = dense_google(r, c, d, t)
    x = t.copy()
    for it in range(1, 9):
        x = G @ x
        o = oracle.pagerank(r, c, d=d, iters=it)
        np.testing.assert_allclose(o.x, x, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", [7, 8])
def test_dense_power_iteration_with_teleport_vector(seed):
    n, d = 48, 0.85
    r, c = random_digraph(n, 0.08, seed)
    rng = np.random.default_rng(seed)
    t = rng.random(n)
    t[rng.random(n) < 0.5] = 0
    t /= t.sum()
    G = dense_google(r, c, d, t)
    x = t.copy()
    for it in range(1, 6):
        x = G @ x
    o = oracle.pagerank(r, c, d=d, iters=5, tele=t, x0=t)
    np.testing.assert_allclose(o.x, x, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_fixed_point_matches_linear_solve(seed):
    """(I - d(M + t delta^T)) x = (1-d) t for sum(x) = 1; the converged
    iterate lies within d*res/(1-d) of it in L1."""
    n, d = 60, 0.85
    r, c = random_digraph(n, 0.07, seed)
    t = np.full(n, 1.0 / n)
    G = dense_google(r, c, d, t)
    A = np.eye(n) - (G - (1 - d) * np.outer(t, np.ones(n)))
    xs = np.linalg.solve(A, (1 - d) * t)
    o = oracle.pagerank(r, c, d=d, iters=1000, tol=1e-13)
    assert o.converged
    assert np.abs(o.x - xs).sum() <= d * o.resid / (1 - d) + 1e-13


def test_residual_contracts_by_d():
    r, c = graphgen.rmat(12, 16, seed=3, relabel="random")
    for d in (0.5, 0.85):
        h = oracle.pagerank(r, c, d=d, iters=30).res_hist
        assert np.all(h[1:] <= d * h[:-1] * (1 + 1e-9) + 1e-17)


def test_tolerance_stops_at_first_residual_below():
    r, c = graphgen.rmat(10, 16, seed=4)
    o = oracle.pagerank(r, c, iters=200, tol=1e-6)
    assert o.converged and o.res_hist[-1] < 1e-6 and np.all(o.res_hist[:-1] >= 1e-6)
    full = oracle.pagerank(r, c, iters=o.iters)
    np.testing.assert_array_equal(full.x, o.x)
    assert not oracle.pagerank(r, c, iters=3, tol=1e-12).converged


# ----------------------------------------------------- personalised PageRank

def test_ppr_on_cycle_closed_form():
    """Teleport to s only on a directed n-cycle: x(s+l) = d^l x(s) and
    x(s) = (1-d) + d^n x(s), so x(s+l) = (1-d) d^l / (1-d^n)."""
    n, d, s = 13, 0.85, 4
    r, c = csr(n, [(i, (i + 1) % n) for i in range(n)])
    o = oracle.ppr(r, c, [s], d=d, iters=2000, tol=1e-15)
    ell = (np.arange(n) - s) % n
    want = (1 - d) * d ** ell / (1 - d ** n)
    assert np.abs(o.x - want).sum() <= d * o.resid / (1 - d) + 1e-14


def test_ppr_on_all_nodes_is_plain_pagerank():
    r, c = graphgen.rmat(9, 8, seed=6)
    n = len(r) - 1
    a = oracle.ppr(r, c, np.arange(n), iters=12).x
    b = oracle.pagerank(r, c, iters=12).x
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-16)


def test_transposed_adjacency_is_the_in_neighbour_lists():
    """transpose() gives every node its in-neighbours, sources ascending
    (brute force over the edge list), and runs on it equal runs that form
    the lists themselves, for plain and personalised PageRank."""
    r, c = graphgen.rmat(10, 8, seed=8)
    n = len(r) - 1
    T = oracle.transpose(r, c)
    src = np.repeat(np.arange(n), np.diff(r))
    for v in range(0, n, 37):
        want = np.sort(src[c == v])
        np.testing.assert_array_equal(T.in_src[T.in_off[v]:T.in_off[v + 1]], want)
    assert T.in_off[n] == len(c)
    a, b = oracle.pagerank(r, c, iters=9), oracle.pagerank(r, c, iters=9, transposed=T)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.res_hist, b.res_hist)
    seeds = np.array([3, 70, 500])
    np.testing.assert_array_equal(oracle.ppr(r, c, seeds, iters=7).x, oracle.ppr(r, c, seeds, iters=7, transposed=T).x)
    r2, c2 = graphgen.rmat(10, 8, seed=9)
    with pytest.raises(ValueError):
        oracle.pagerank(r2, c2, iters=2, transposed=T)


# ---------------------------------------------------------------- PNG layout

def brute_png(row_off, col, q):
    """The layout written directly as set-builder expressions."""
    n = len(row_off) - 1
    k = -(-n // q)
    N = [set(col[row_off[u]:row_off[u + 1]].tolist()) for u in range(n)]
    P = [range(p * q, min(n, (p + 1) * q)) for p in range(k)]
    U = [[[u for u in P[p] if any(v // q == pp for v in N[u])] for pp in range(k)] for p in range(k)]
    png_off = np.array([[sum(len(U[p][j]) for j in range(jj)) for jj in range(k + 1)]
                        for p in range(k)])
    png_src = [u for p in range(k) for pp in range(k) for u in U[p][pp]]
    upd_start = [sum(len(U[p][j]) for j in range(jj) for p in range(k)) for jj in range(k + 1)]
    wo = np.array([[sum(len(U[p2][pp]) for p2 in range(p)) for pp in range(k)] for p in range(k)])
    bins = []
    for pp in range(k):
        b = []
        for p in range(k):
            for u in U[p][pp]:
                vs = sorted(v for v in N[u] if v // q == pp)
                b += [v | (0x80000000 if i == 0 else 0) for i, v in enumerate(vs)]
        bins.append(b)
    did_start = [sum(len(bins[j]) for j in range(jj)) for jj in range(k + 1)]
    did = [x for b in bins for x in b]
    return dict(png_off=png_off, png_src=png_src, upd_start=upd_start, wo=wo,
                did_start=did_start, did=did, k=k)


def assert_png_equal(o, b):
    assert o.k == b["k"]
    np.testing.assert_array_equal(o.png_off, b["png_off"])
    np.testing.assert_array_equal(o.png_src, np.asarray(b["png_src"], dtype=np.int32))
    np.testing.assert_array_equal(o.upd_start, b["upd_start"])
    np.testing.assert_array_equal(o.wo, b["wo"])
    np.testing.assert_array_equal(o.did_start, b["did_start"])
    np.testing.assert_array_equal(o.did, np.asarray(b["did"], dtype=np.uint32))


def test_sec3_1_worked_example_write_offsets():
    g = json.load(open(os.path.join(GOLDEN, "sec3_1_write_offsets.json")))
    r, c = csr(g["n"], g["edges"])
    o = oracle.png_layout(r, c, g["q"])
    assert o.wo[2].tolist() == g["expected"]["wo_row_of_partition_2"]
    assert_png_equal(o, brute_png(r, c, g["q"]))


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
@pytest.mark.parametrize("q", [1, 2, 3, 4, 8, 16, 64])
def test_png_matches_set_definitions(seed, q):
    n = [9, 33, 64, 50][seed - 1]
    r, c = random_digraph(n, 0.15, seed, dangling_frac=0.25)
    assert_png_equal(oracle.png_layout(r, c, q), brute_png(r, c, q))


def test_png_extremes_and_invariants():
    r, c = graphgen.rmat(11, 16, seed=9, relabel="random")
    n, m = len(r) - 1, len(c)
    nondangling = int((np.diff(r) > 0).sum())
    assert oracle.png_layout(r, c, 1).eprime == m          # q = 1: nothing compresses
    assert oracle.png_layout(r, c, n).eprime == nondangling  # one partition
    for q in (16, 128, 512):
        o = oracle.png_layout(r, c, q)
        assert o.did_start[-1] == m
        flags = (o.did >> 31).astype(np.int64)
        assert flags.sum() == o.eprime == o.upd_start[-1]
        rr = m / o.eprime
        assert 1.0 <= rr <= m / nondangling
        for pp in range(o.k):
            ids = o.did[o.did_start[pp]:o.did_start[pp + 1]] & 0x7FFFFFFF
            assert np.all(ids // q == pp)
            if len(ids):
                assert o.did[o.did_start[pp]] >> 31 == 1


@pytest.mark.parametrize("q", [1, 3, 64, 256, 4096])
def test_pcpm_route_equals_pull_route(q):
    """Alg. 3 + Alg. 5 over the layout reproduce Eq. 1 (they reorder the sum)."""
    r, c = graphgen.rmat(12, 16, seed=21, relabel="random")
    n = len(r) - 1
    o = oracle.png_layout(r, c, q)
    x = oracle.pagerank(r, c, iters=3).x
    y_pull = oracle.pagerank(r, c, iters=4).x
    y_pcpm, res = oracle.pcpm_iterate(r, o, x)
    np.testing.assert_allclose(y_pcpm, y_pull, rtol=0, atol=1e-15)
    assert abs(res - np.abs(y_pull - x).sum()) < 1e-15


def test_literal_alg5_pointer_is_off_by_one():
    """Alg. 5 as printed starts the update pointer at 0 and advances it before
    the read, so the first destination ID of a bin would take the bin's second
    update and the last message would read past the bin.  The reading used
    here (start one before the bin) reproduces the pull result."""
    g = json.load(open(os.path.join(GOLDEN, "sec3_1_write_offsets.json")))
    r, c = csr(g["n"], g["edges"])
    o = oracle.png_layout(r, c, g["q"])
    x = np.arange(1, g["n"] + 1, dtype=np.float64)
    x /= x.sum()
    y, _ = oracle.pcpm_iterate(r, o, x)
    np.testing.assert_allclose(y, oracle.pagerank(r, c, iters=1, x0=x).x, rtol=0, atol=1e-16)
    # bin 2 holds two messages (from nodes 0 and 8): 6*,7,6*,7 with 2 updates
    ids = o.did[o.did_start[2]:o.did_start[3]]
    nupd = int(o.upd_start[3] - o.upd_start[2])
    assert nupd == 2 and (ids >> 31).tolist() == [1, 0, 1, 0]
    literal = np.cumsum(ids >> 31)          # pointer after "+= MSB", from 0
    assert literal.max() == nupd            # one past the last update
    assert (literal - 1).tolist() == [0, 0, 1, 1]


# ------------------------------------------ the pins reject plausible mistakes

def _wrong_pagerank(r, c, d, iters, mistake):
    n = len(r) - 1
    x = np.full(n, 1.0 / n)
    od = np.diff(r)
    for _ in range(iters):
        spr = np.where(od > 0, x / np.maximum(od, 1), 0.0)
        s = np.zeros(n)
        src = np.repeat(np.arange(n), od)
        if mistake == "transposed":
            np.add.at(s, src, spr[c])
        else:
            np.add.at(s, c, spr[src])
        D = x[od == 0].sum()
        if mistake == "no_dangling":
            D = 0.0
        if mistake == "no_jump":
            x = d * (s + D / n)
        elif mistake == "divide_by_indegree":
            indeg = np.bincount(c, minlength=n)
            s = np.zeros(n)
            np.add.at(s, c, x[src] / np.maximum(indeg[c], 1))
            x = (1 - d) / n + d * (s + D / n)
        else:
            x = (1 - d) / n + d * (s + D / n)
    return x


@pytest.mark.parametrize("mistake", ["transposed", "no_dangling", "no_jump", "divide_by_indegree"])
def test_pins_catch_planted_mistakes(mistake):
    """A plausible mistake in the recurrence fails at least one pin."""
    d = 0.85
    failed = []
    n = 5
    for name, edges, want0 in [
        ("in_star", [(i, 0) for i in range(1, n)], (1 + (n - 1) * d) / (n + (n - 1) * d)),
        ("out_star", [(0, i) for i in range(1, n)], 1.0 / (n + d)),
        ("bi_star", [(0, i) for i in range(1, n)] + [(i, 0) for i in range(1, n)],
         (1 + (n - 1) * d) / (n * (1 + d))),
    ]:
        r, c = csr(n, edges)
        x = _wrong_pagerank(r, c, d, 400, mistake)
        if abs(x[0] - want0) > 1e-9 or abs(x.sum() - 1) > 1e-9:
            failed.append(name)
    r, c = random_digraph(30, 0.1, 3)
    G = dense_google(r, c, d, np.full(30, 1 / 30))
    x = np.full(30, 1 / 30)
    for _ in range(5):
        x = G @ x
    if np.abs(_wrong_pagerank(r, c, d, 5, mistake) - x).max() > 1e-12:
        failed.append("dense")
    assert failed, f"no pin rejects the mistake {mistake}"
    # and the correct recurrence passes the same checks
    assert np.abs(_wrong_pagerank(r, c, d, 5, "none") - x).max() < 1e-14


# ------------------------------------------------ one step at chosen nodes

@pytest.mark.parametrize("seed,n,p,d,use_tele", [(11, 30, 0.2, 0.85, False), (12, 64, 0.07, 0.6, True),
                                                 (13, 9, 0.4, 0.85, False)])
def test_step_at_matches_dense_google_product(seed, n, p, d, use_tele):
    """A step from an arbitrary (not normalised) vector, at a random subset of
    nodes, equals rows of the dense Google matrix times that vector."""
    r, c = random_digraph(n, p, seed)
    rng = np.random.default_rng(seed)
    if use_tele:
        t = rng.random(n)
        t[rng.random(n) < 0.5] = 0
        t /= t.sum()
    else:
        t = np.full(n, 1.0 / n)
    x = rng.random(n)
    want = dense_google(r, c, d, t) @ x
    # the dangling spread uses the dangling mass of x, and the jump (1-d) t
    # weighs the mass of x in the dense form: correct that term for sum(x) != 1
    want += (1 - d) * t * (1.0 - x.sum())
    nodes = rng.choice(n, size=max(1, n // 3), replace=False)
    got = oracle.step_at(r, c, x, nodes, d=d, tele=t if use_tele else None, threads=3)
    np.testing.assert_allclose(got, want[nodes], rtol=0, atol=1e-14)
    # all nodes, any thread count, equal one full iteration of the pull oracle
    full = oracle.step_at(r, c, x, np.arange(n), d=d, tele=t if use_tele else None, threads=1)
    np.testing.assert_allclose(full, want, rtol=0, atol=1e-14)


def test_step_at_rejects_bad_node_lists():
    r, c = random_digraph(10, 0.3, 1)
    with pytest.raises(ValueError):
        oracle.step_at(r, c, np.ones(10) / 10, [3, 3])
    with pytest.raises(ValueError):
        oracle.step_at(r, c, np.ones(10) / 10, [10])
    assert oracle.step_at(r, c, np.ones(10) / 10, []).shape == (0,)
