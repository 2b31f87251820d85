"""Parity at the workloads' full sizes, in the configurations bench.py times.

* RMAT-24 (EF 16, seed 2), random and in-degree labels (from the generator,
  and from pcpm_relabel as bench.py runs it), q = 16384, to L1 residual 1e-6:
  whole vectors against the FP64 oracle at the same iteration count.
* The paper-scale graphs (RMAT-26 EF 24 seed 3, random labels; uniform graph
  of 50M nodes and 1B draws, seed 4), 20 iterations from the uniform start:
  the whole 20th iterate against the oracle's, the residual history against
  the oracle's, one oracle step from the GPU's 19th iterate at sampled
  nodes, unit mass and residuals contracting by d.
* Batched personalised PageRank on RMAT-22 (EF 16, seed 5) with 8/32/64 seed
  sets at the autotuned partition size (every vector against the oracle),
  and the 16-graph uneven batch.
* The learned warm start on a held-out RMAT-24 graph.
* The weighted SpMV on RMAT-24 in both update orders.
* The in-degree relabelling of RMAT-26 EF 24: permutation and row offsets
  against the oracle's, sampled rows, and the compression ratio it buys.
"""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1709_07122_amd")

pytestmark = [pytest.mark.gpu, pytest.mark.full]

D = 0.85


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_vector(got, ref, l1_tol=1e-5, rel_tol=1e-3):
    got = got.astype(np.float64)
    n = len(ref)
    l1 = np.abs(got - ref).sum()
    assert l1 <= l1_tol, l1
    big = ref > 1.0 / n
    assert big.any()
    rel = (np.abs(got - ref)[big] / ref[big]).max()
    assert rel <= rel_tol, rel


@pytest.mark.parametrize("relabel", ["random", "indegree", "pcpm_relabel"])
def test_rmat24_to_tolerance(relabel):
    if relabel == "pcpm_relabel":  # the random-labelled graph put in in-degree order on the GPU (bench.py)
        r, c = graphgen.rmat(24, 16, seed=2, relabel="random")
        _, ro, co = P.relabel(dev(r), dev(c), key="in")
        r, c = ro.cpu().numpy(), co.cpu().numpy()
        del ro, co
    else:
        r, c = graphgen.rmat(24, 16, seed=2, relabel=relabel)
    png = P.build_png(dev(r), dev(c), part_log2=14)
    res = P.pagerank(png, d=D, tol=1e-6, max_iters=100)
    png.close()
    assert res.converged and res.resid < 1e-6
    o = oracle.pagerank(r, c, d=D, iters=res.iters)
    check_vector(res.pr.cpu().numpy(), o.x)
    # the oracle sees the same stopping point
    assert o.res_hist[-1] < 1.05e-6 and o.res_hist[-2] >= 0.95e-6


def sample_nodes(r, c, count, seed):
    """Largest in-degrees, the last nodes (ragged tail), node 0 and random ones."""
    n = len(r) - 1
    indeg = np.bincount(c, minlength=n)
    top = np.argpartition(indeg, -256)[-256:]
    rng = np.random.default_rng(seed)
    pick = np.concatenate([top, np.arange(n - 64, n), [0], rng.choice(n, count, replace=False)])
    return np.unique(pick)


@pytest.mark.parametrize("kind", ["rmat26_ef24", "uniform_50m_1b"])
def test_paper_scale_twenty_iterations(kind):
    """20 iterations from the uniform start (the paper's protocol): the whole
    20th iterate against the oracle's 20th (L1 and relative error), one
    oracle step from the GPU's own 19th iterate at sampled nodes, unit mass
    and residuals contracting by d."""
    if kind == "rmat26_ef24":
        r, c = graphgen.rmat(26, 24, seed=3, relabel="random")
    else:
        r, c = graphgen.uniform(50_000_000, 1_000_000_000, seed=4)
    n = len(r) - 1
    print(f"[{kind}] n={n} m={len(c)}", flush=True)
    png = P.build_png(dev(r), dev(c), part_log2=14)
    res19 = P.pagerank(png, d=D, tol=0.0, max_iters=19, want_hist=True)
    x20, _ = P.iterate(png, res19.pr, d=D)
    res20 = P.pagerank(png, d=D, tol=0.0, max_iters=20, want_hist=True)
    png.close()
    x19 = res19.pr.cpu().numpy()
    y = x20.cpu().numpy()
    y20 = res20.pr.cpu().numpy()
    del res19, x20, res20.pr
    torch.cuda.empty_cache()
    # pcpm_pagerank's 20th iterate and pcpm_iterate from its 19th agree up to
    # the FP32 rounding of the output (their FP64 dangling sums are formed in
    # different orders)
    assert np.all(np.abs(y20.astype(np.float64) - y) <= 2.0 ** -22 * np.abs(y.astype(np.float64)))
    nodes = sample_nodes(r, c, 20000, seed=n % 1000)
    ref = oracle.step_at(r, c, x19.astype(np.float64), nodes, d=D)
    rel = np.abs(y[nodes].astype(np.float64) - ref) / ref
    assert rel.max() <= 1e-5, rel.max()
    del x19, y
    assert abs(y20.astype(np.float64).sum() - 1.0) <= 1e-5
    h = res20.res_hist
    assert len(h) == 20 and np.all(np.isfinite(h))
    assert np.all(h[1:] <= D * h[:-1] * 1.001 + 1e-7), h
    # the whole vector: the oracle runs the same 20 iterations from the same
    # uniform start
    o = oracle.pagerank(r, c, d=D, iters=20)
    print(f"[{kind}] oracle {o.sec_per_iter * 1e3:.0f} ms/iteration", flush=True)
    check_vector(y20, o.x)
    # the GPU's FP64 residuals follow the oracle's: each GPU iterate lies
    # within 3 * 2^-24 / (1 - d) of the oracle's in L1 (FP32 roundings of the
    # start vector, of PR/outdeg and of each output, each at most 2^-24 of a
    # unit-mass vector, carried through a contraction by d), and a residual
    # involves two iterates
    np.testing.assert_allclose(h, o.res_hist, rtol=0, atol=2 * 3 * 2.0 ** -24 / (1 - D))


@pytest.fixture(scope="module")
def rmat22():
    return graphgen.rmat(22, 16, seed=5, relabel="random")


@pytest.fixture(scope="module")
def rmat22_transposed(rmat22):
    return oracle.transpose(*rmat22)


@pytest.mark.parametrize("k", [8, 32, 64])
def test_ppr_rmat22_autotuned(rmat22, rmat22_transposed, k):
    """Every one of the k vectors against the oracle at its own iteration
    count."""
    from paper_1709_07122_amd import autotune

    r, c = rmat22
    n = len(r) - 1
    rt, ct = dev(r), dev(c)
    tune = autotune.tune(rt, ct, vectors=k, cache=None)
    png = P.build_png(rt, ct, part_log2=tune.part_log2, update_order=tune.update_order)
    off, seeds = graphgen.seed_sets(n, k, seed=k)
    res = P.ppr_batch(png, off, seeds, d=D, tol=1e-6, max_iters=200)
    png.close()
    assert res.converged and np.all(res.resid < 1e-6)
    x = res.pr.cpu().numpy()
    np.testing.assert_allclose(x.astype(np.float64).sum(axis=0), 1.0, atol=1e-5)
    for j in range(k):
        ref = oracle.ppr(r, c, seeds[off[j]:off[j + 1]], d=D, iters=int(res.iters[j]),
                         transposed=rmat22_transposed).x
        check_vector(x[:, j], ref)


@pytest.mark.parametrize("part_log2", [12, 14])
def test_sixteen_uneven_graphs(part_log2):
    graphs, shapes = graphgen.uneven_rmat_batch(16, seed=100)
    r, c, off, sizes = P.union_csr(graphs, part_log2)
    png = P.build_png(dev(r), dev(c), part_log2=part_log2, graph_node_off=off, graph_nodes=sizes)
    res = P.pagerank(png, d=D, tol=1e-6, max_iters=200)
    it, resid = png.graph_results()
    png.close()
    assert res.converged and np.all(resid < 1e-6)
    x = res.pr.cpu().numpy()
    for g, (rg, cg) in enumerate(graphs):
        ref = oracle.pagerank(rg, cg, d=D, iters=int(it[g])).x
        check_vector(x[off[g]:off[g] + sizes[g]], ref)
        assert np.all(x[off[g] + sizes[g]:off[g + 1]] == 0.0)


def test_warm_start_on_held_out_rmat24():
    ws = P.warmstart
    r, c = graphgen.rmat(24, 16, seed=2000, relabel="random")
    png = P.build_png(dev(r), dev(c), part_log2=14)
    pr0, fallback = ws.warm_start(png, ws.load(ws.DEFAULT_WEIGHTS), d=D)
    assert not fallback
    cold = P.pagerank(png, d=D, tol=1e-6, max_iters=100)
    warm = P.pagerank(png, d=D, tol=1e-6, max_iters=100, init=pr0)
    png.close()
    assert cold.converged and warm.converged
    assert warm.iters <= cold.iters - 3, (warm.iters, cold.iters)
    star = oracle.pagerank(r, c, d=D, iters=300, tol=1e-11).x
    for res in (cold, warm):
        err = np.abs(res.pr.cpu().numpy().astype(np.float64) - star).sum()
        assert err <= D * res.resid / (1 - D) + 1e-5, err


@pytest.mark.parametrize("update_order", [1, 2])
def test_weighted_spmv_rmat24(update_order):
    """SpMV (Sec. 3.5) on RMAT-24 with weights uniform in [-1, 1), in both
    update orders, against the FP64 oracle within the bound of pcpm_spmv."""
    r, c = graphgen.rmat(24, 16, seed=2, relabel="random")
    n = len(r) - 1
    rng = np.random.default_rng(1002)
    w = rng.uniform(-1.0, 1.0, len(c)).astype(np.float32)
    x = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    png = P.build_png(dev(r), dev(c), part_log2=14, weights=dev(w), update_order=update_order)
    y = P.spmv(png, dev(x)).cpu().numpy().astype(np.float64)
    png.close()
    ref = oracle.spmv(r, c, x, w)
    aw = np.abs(w.astype(np.float64))
    xmax = float(np.abs(x).max())
    indeg = np.bincount(c, minlength=n)
    wcol = float(np.bincount(c, weights=aw, minlength=n).max())
    s = min(50 - int(np.ceil(np.log2(aw.max() * xmax))), 62 - int(np.ceil(np.log2(wcol * xmax)))) - 1
    bound = indeg * 2.0 ** -s + 2.0 ** -23 * np.abs(ref) + 2.0 ** -150
    assert np.all(np.abs(y - ref) <= bound)


def test_relabel_rmat26_indegree():
    """pcpm_relabel on 1.58B edges: the permutation and row offsets exactly as
    the oracle's degree order gives them (in-degrees from the oracle's own
    count), 2000 sampled rows exactly, every row strictly ascending, and r of
    the relabelled PNG above the random labelling's."""
    r, c = graphgen.rmat(26, 24, seed=3, relabel="random")
    n = len(r) - 1
    rd, cd = dev(r), dev(c)
    perm, ro2, c2 = P.relabel(rd, cd, key="in")
    perm, ro2 = perm.cpu().numpy(), ro2.cpu().numpy()
    deg = np.bincount(c, minlength=n)
    order = np.lexsort((np.arange(n), -deg))
    want = np.empty(n, np.int64)
    want[order] = np.arange(n)
    np.testing.assert_array_equal(perm, want)
    outdeg = np.diff(np.asarray(r, np.int64))
    np.testing.assert_array_equal(np.diff(ro2.astype(np.int64)), outdeg[order])
    c2h = c2.cpu().numpy()
    rng = np.random.default_rng(1)
    for i in rng.choice(n, 2000, replace=False):
        old = order[i]
        row = np.sort(want[np.asarray(c[r[old]:r[old + 1]], np.int64)])
        np.testing.assert_array_equal(c2h[ro2[i]:ro2[i + 1]], row)
    d = np.diff(c2h.astype(np.int64))
    starts = np.zeros(len(c2h), bool)
    starts[ro2[:-1][np.diff(ro2) > 0]] = True
    assert np.all(d[~starts[1:]] > 0)
    del c2h, d, starts
    e_rand = P.build_png(rd, cd).info["eprime"]
    del rd, cd
    e_deg = P.build_png(dev(ro2), c2).info["eprime"]
    assert e_deg < e_rand
