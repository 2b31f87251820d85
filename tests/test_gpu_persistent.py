"""The persistent solve and batch (one cooperative launch per pcpm_pagerank
or pcpm_ppr_batch, grid-wide barriers between the phases, convergence and
vector refills on the device) against one launch per phase: the same
iterations, residuals and ranks bit for bit (integer gather sums, the same
FP64 reductions in the same order), and both against the FP64 oracle; the
bounded device-side waits forced to give up from the host with a tiny spin
limit."""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1709_07122_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def solve(png, mode, **kw):
    png.set_launch(mode)
    return P.pagerank(png, **kw)


def check_vector(got, ref, l1_tol=1e-5, rel_tol=1e-3):
    got = np.asarray(got, np.float64)
    n = len(ref)
    assert np.abs(got - ref).sum() <= l1_tol
    big = ref > 1.0 / n
    if big.any():
        assert (np.abs(got - ref)[big] / ref[big]).max() <= rel_tol


def assert_same(a, b):
    assert a.iters == b.iters and a.converged == b.converged
    np.testing.assert_array_equal(a.res_hist, b.res_hist)
    assert torch.equal(a.pr, b.pr)


CASES = [  # (scale, edge factor, labels, part_log2, scatter_chunk, gather_chunk, update order)
    (15, 16, "random", 14, 0, 0, 0),
    (15, 16, "random", 10, 4096, 4096, 1),   # split pairs and split bins (merge units)
    (15, 16, "indegree", 12, 0, 65536, 2),   # hub bins split, PNG order
    (14, 8, "random", 6, 512, 300, 1),       # 256 partitions, many small merge units
    (13, 12, "indegree", 9, 0, 2048, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-{c[2]}-q{c[3]}-o{c[6]}" for c in CASES])
def test_persistent_equals_per_phase_and_oracle(case):
    scale, ef, labels, pl, sc, gc, order = case
    r, c = graphgen.rmat(scale, ef, seed=31 + scale, relabel=labels)
    png = P.build_png(dev(r), dev(c), part_log2=pl, scatter_chunk=sc, gather_chunk=gc, update_order=order)
    assert png.launch_grid > 0
    if gc:
        assert png.info["split_bins"] > 0
    for tol, iters in ((0.0, 20), (1e-6, 200)):
        a = solve(png, 1, tol=tol, max_iters=iters)
        b = solve(png, 2, tol=tol, max_iters=iters)
        assert_same(a, b)
        ref = oracle.pagerank(r, c, iters=b.iters)
        check_vector(b.pr.cpu().numpy(), ref.x)
    # a start vector of the caller's, and a single iteration
    x0 = torch.rand(png.n, device="cuda") * (2.0 / png.n)
    a = solve(png, 1, tol=0.0, max_iters=1, init=x0.clone())
    b = solve(png, 2, tol=0.0, max_iters=1, init=x0.clone())
    assert_same(a, b)


def test_persistent_multigraph_with_frozen_graphs():
    """Graphs of a batch converge at different iterations; the persistent
    solve keeps each converged graph's iterate exactly as the per-phase one
    does, and every graph matches its own oracle run."""
    rng = np.random.default_rng(9)
    graphs = [graphgen.rmat(int(rng.integers(7, 14)), int(rng.integers(4, 20)), seed=500 + i, relabel="random")
              for i in range(12)]
    r, c, off, sizes = P.union_csr(graphs, 9)
    png = P.build_png(dev(r), dev(c), part_log2=9, graph_node_off=off, graph_nodes=sizes, gather_chunk=4096)
    a = solve(png, 1, tol=1e-7, max_iters=300)
    it_a, res_a = png.graph_results()
    b = solve(png, 2, tol=1e-7, max_iters=300)
    it_b, res_b = png.graph_results()
    assert_same(a, b)
    np.testing.assert_array_equal(it_a, it_b)
    np.testing.assert_array_equal(res_a, res_b)
    assert len(set(it_b.tolist())) > 1  # the graphs really stop at different iterations
    x = b.pr.cpu().numpy()
    for g, (rg, cg) in enumerate(graphs):
        check_vector(x[off[g]:off[g] + sizes[g]], oracle.pagerank(rg, cg, iters=int(it_b[g])).x)
        assert np.all(x[off[g] + sizes[g]:off[g + 1]] == 0.0)


def test_default_mode_and_modes_are_checked():
    r, c = graphgen.rmat(10, 8, seed=3)
    png = P.build_png(dev(r), dev(c), part_log2=7)
    base = P.pagerank(png, tol=0.0, max_iters=7)  # mode 0: one launch per phase
    assert_same(base, solve(png, 2, tol=0.0, max_iters=7))
    assert_same(base, solve(png, 0, tol=0.0, max_iters=7))
    for bad in (-1, 3):
        with pytest.raises(P.PCPMError) as ei:
            png.set_launch(bad)
        assert ei.value.status == P.PCPM_ERR_INVALID_ARG


def test_bounded_waits_give_up_with_an_error():
    """A spin limit of one poll makes the workgroups that wait at the first
    grid barrier give up: the solve ends with PCPM_ERR_DEVICE instead of
    hanging, and the next solve with the default limit is exact again."""
    r, c = graphgen.rmat(14, 16, seed=41, relabel="random")
    png = P.build_png(dev(r), dev(c), part_log2=10, gather_chunk=8192)
    png.set_launch(2, spin_limit=1)
    with pytest.raises(P.PCPMError) as ei:
        P.pagerank(png, tol=0.0, max_iters=5)
    assert ei.value.status == P.PCPM_ERR_DEVICE
    assert "limit" in str(ei.value)
    b = solve(png, 2, tol=0.0, max_iters=5)
    assert_same(solve(png, 1, tol=0.0, max_iters=5), b)
    check_vector(b.pr.cpu().numpy(), oracle.pagerank(r, c, iters=5).x)


PPR_CASES = [  # (part_log2, gather_chunk, update order, k vectors)
    (12, 0, 1, 3),       # one tile, no refills
    (12, 0, 2, 11),      # tiles of 4 with refills, PNG order
    (10, 2048, 1, 37),   # split bins (merge units), tiles of 16
    (13, 4096, 2, 9),    # tiles of 2, split bins, PNG order
]


@pytest.mark.parametrize("case", PPR_CASES, ids=[f"q{c[0]}-g{c[1]}-o{c[2]}-k{c[3]}" for c in PPR_CASES])
def test_persistent_ppr_batch_equals_per_phase_and_oracle(case):
    pl, gc, order, k = case
    r, c = graphgen.rmat(14, 12, seed=77, relabel="random")
    n = len(r) - 1
    png = P.build_png(dev(r), dev(c), part_log2=pl, gather_chunk=gc, update_order=order)
    if gc:
        assert png.info["split_bins"] > 0
    off, seeds = graphgen.seed_sets(n, k, seed=k)
    png.set_launch(1)
    a = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=200)
    png.set_launch(2)
    b = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=200)
    assert a.converged and b.converged
    np.testing.assert_array_equal(a.iters, b.iters)
    np.testing.assert_array_equal(a.resid, b.resid)
    assert torch.equal(a.pr, b.pr)
    x = b.pr.cpu().numpy()
    T = oracle.transpose(r, c)
    for j in range(k):
        check_vector(x[:, j], oracle.ppr(r, c, seeds[off[j]:off[j + 1]], iters=int(b.iters[j]), transposed=T).x)


def test_persistent_ppr_bounded_waits_give_up():
    r, c = graphgen.rmat(13, 8, seed=78, relabel="random")
    n = len(r) - 1
    png = P.build_png(dev(r), dev(c), part_log2=11)
    off, seeds = graphgen.seed_sets(n, 9, seed=3)
    png.set_launch(2, spin_limit=1)
    with pytest.raises(P.PCPMError) as ei:
        P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=50)
    assert ei.value.status == P.PCPM_ERR_DEVICE
    png.set_launch(2)
    b = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=200)
    png.set_launch(1)
    a = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=200)
    assert torch.equal(a.pr, b.pr)
