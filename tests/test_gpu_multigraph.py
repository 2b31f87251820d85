"""Several graphs of uneven size in one handle: each graph runs its own
PageRank (own n, jump, dangling spread, residual and convergence), checked
graph by graph against the FP64 oracle run on that graph alone."""
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


def uneven_batch(count, seed):
    rng = np.random.default_rng(seed)
    graphs = []
    for i in range(count):
        scale = int(rng.integers(6, 13))
        ef = int(rng.integers(4, 17))
        graphs.append(graphgen.rmat(scale, ef, seed=1000 + seed * 100 + i, relabel="random"))
    return graphs


def build_union(graphs, part_log2, **kw):
    r, c, off, sizes = P.union_csr(graphs, part_log2)
    png = P.build_png(torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda(), part_log2=part_log2,
                      graph_node_off=off, graph_nodes=sizes, **kw)
    return png, off, sizes


def check_slices(x, graphs, off, sizes, iters):
    for g, (r, c) in enumerate(graphs):
        ref = oracle.pagerank(r, c, iters=int(iters[g])).x
        got = x[off[g]:off[g] + sizes[g]].astype(np.float64)
        assert np.abs(got - ref).sum() <= 1e-5, g
        big = ref > 1.0 / len(ref)
        assert (np.abs(got - ref)[big] / ref[big]).max() <= 1e-3, g
        assert np.all(x[off[g] + sizes[g]:off[g + 1]] == 0.0)  # padding


@pytest.mark.parametrize("part_log2", [6, 9, 12])
def test_sixteen_graphs_fixed_iterations(part_log2):
    graphs = uneven_batch(16, seed=1)
    png, off, sizes = build_union(graphs, part_log2)
    assert png.info["num_graphs"] == 16
    res = P.pagerank(png, tol=0.0, max_iters=20)
    it, _ = png.graph_results()
    assert np.all(it == 20)
    check_slices(res.pr.cpu().numpy(), graphs, off, sizes, it)


def test_sixteen_graphs_converge_separately():
    graphs = uneven_batch(16, seed=2)
    png, off, sizes = build_union(graphs, 7, gather_chunk=4096)  # split bins too
    res = P.pagerank(png, tol=1e-6, max_iters=300)
    assert res.converged
    it, rs = png.graph_results()
    assert np.all(rs < 1e-6)
    assert it.max() == res.iters and len(set(it.tolist())) > 1  # graphs stop at different iterations
    check_slices(res.pr.cpu().numpy(), graphs, off, sizes, it)
    # each graph stopped at the first iteration whose FP64 residual fell below
    # tol; the oracle's residual one iteration earlier was not yet below it
    for g, (r, c) in enumerate(graphs):
        h = oracle.pagerank(r, c, iters=int(it[g])).res_hist
        assert h[-1] < 1.2e-6 and (len(h) == 1 or h[-2] > 0.8e-6), g


def test_union_validation():
    a = graphgen.rmat(6, 4, seed=1)
    b = graphgen.rmat(6, 4, seed=2)
    r, c, off, sizes = P.union_csr([a, b], 6)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    # an edge from graph 0 into graph 1
    c_bad = c.copy()
    c_bad[0] = off[1] + 1 if c_bad[0] != off[1] + 1 else off[1] + 2
    rows = np.repeat(np.arange(len(r) - 1), np.diff(r))
    c_bad[: r[rows[0] + 1]] = np.sort(c_bad[: r[rows[0] + 1]])
    with pytest.raises(P.PCPMError) as ei:
        P.build_png(dev(r), dev(c_bad), part_log2=6, graph_node_off=off, graph_nodes=sizes)
    assert ei.value.status == P.PCPM_ERR_GRAPH
    # offsets that are not multiples of q
    with pytest.raises(P.PCPMError) as ei:
        P.build_png(dev(r), dev(c), part_log2=7, graph_node_off=off, graph_nodes=sizes)
    assert ei.value.status == P.PCPM_ERR_INVALID_ARG
