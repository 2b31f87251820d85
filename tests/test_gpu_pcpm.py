"""GPU parity: libpcpm (through its C ABI) against the FP64 CPU oracle.

* layout: bit-exact against the oracle's canonical PNG,
* ranks: L1 distance <= 1e-5 and max relative error <= 1e-3 on nodes whose
  rank exceeds 1/n, after the same number of iterations from the same start,
* residuals: FP64 on the device, compared with the oracle's FP64 residual of
  the FP64 iterates (they differ by the FP32 rounding of the ranks).
"""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1709_07122_amd")

pytestmark = pytest.mark.gpu

L1_TOL = 1e-5
REL_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def build(r, c, **kw):
    return P.build_png(dev(r), dev(c), **kw)


def csr(n, edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return graphgen.from_edges(n, e[:, 0], e[:, 1], threads=1)


def random_digraph(n, p, seed, dangling_frac=0.3):
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < p
    np.fill_diagonal(a, False)
    a[rng.random(n) < dangling_frac, :] = False
    u, v = np.nonzero(a)
    return csr(n, np.stack([u, v], 1))


def assert_layout_equal(png, r, c, part_log2):
    got = png.export()
    want = oracle.png_layout(r, c, 1 << part_log2)
    assert png.info["k"] == want.k and png.info["eprime"] == want.eprime
    np.testing.assert_array_equal(got["png_off"], want.png_off)
    np.testing.assert_array_equal(got["upd_start"], want.upd_start)
    np.testing.assert_array_equal(got["wo"], want.wo)
    np.testing.assert_array_equal(got["did_start"], want.did_start)
    np.testing.assert_array_equal(got["png_src"], want.png_src)
    np.testing.assert_array_equal(got["did"], want.did)


def assert_ranks_close(x_gpu, x_ref):
    x_gpu = np.asarray(x_gpu, dtype=np.float64)
    n = len(x_ref)
    l1 = np.abs(x_gpu - x_ref).sum()
    big = x_ref > 1.0 / n
    rel = (np.abs(x_gpu - x_ref)[big] / x_ref[big]).max() if big.any() else 0.0
    assert l1 <= L1_TOL, f"L1 {l1:.3e}"
    assert rel <= REL_TOL, f"max rel {rel:.3e}"
    return l1, rel


# ------------------------------------------------------------------ layout

@pytest.mark.parametrize("seed,n,part_log2", [(1, 9, 1), (2, 33, 2), (3, 64, 3), (4, 50, 4), (5, 64, 6)])
def test_layout_small_random(seed, n, part_log2):
    r, c = random_digraph(n, 0.15, seed, dangling_frac=0.25)
    assert_layout_equal(build(r, c, part_log2=part_log2), r, c, part_log2)


@pytest.mark.parametrize("relabel", [None, "random", "indegree"])
@pytest.mark.parametrize("part_log2", [5, 9, 12])
def test_layout_rmat12(relabel, part_log2):
    r, c = graphgen.rmat(12, 16, seed=7, relabel=relabel)
    assert_layout_equal(build(r, c, part_log2=part_log2), r, c, part_log2)


@pytest.mark.parametrize("part_log2", [8, 14])
def test_layout_rmat16(part_log2):
    """RMAT scale 16, edge factor 16 (65,536 nodes), random labels."""
    r, c = graphgen.rmat(16, 16, seed=1, relabel="random")
    assert_layout_equal(build(r, c, part_log2=part_log2), r, c, part_log2)


@pytest.mark.parametrize("relabel,part_log2,chunk", [("indegree", 8, 64), ("indegree", 10, 1000),
                                                     (None, 5, 1), ("random", 7, 333)])
def test_layout_with_small_build_chunks(relabel, part_log2, chunk):
    """Count and fill split every partition's edges into many chunks (the
    paths that skewed graphs take at full size); the layout is the same."""
    r, c = graphgen.rmat(12, 16, seed=11, relabel=relabel)
    png = build(r, c, part_log2=part_log2, build_chunk=chunk)
    assert_layout_equal(png, r, c, part_log2)
    res = P.pagerank(png, tol=0.0, max_iters=12)
    assert_ranks_close(res.pr.cpu().numpy(), oracle.pagerank(r, c, iters=12).x)


def test_layout_ragged_and_degenerate():
    # n not a multiple of q, plus a hub row longer than one wavefront
    n = 1000
    rng = np.random.default_rng(3)
    e = [(0, v) for v in range(1, 900)] + [(int(a), int(b)) for a, b in rng.integers(0, n, (5000, 2))]
    r, c = csr(n, e)
    for pl in (3, 7, 10):
        assert_layout_equal(build(r, c, part_log2=pl), r, c, pl)
    # a single node, no edges
    r, c = csr(1, np.zeros((0, 2)))
    png = build(r, c, part_log2=4)
    assert png.info["eprime"] == 0 and png.info["k"] == 1


# ------------------------------------------------------------------ ranks

def test_one_iteration_matches_oracle():
    r, c = graphgen.rmat(14, 16, seed=2, relabel="random")
    n = len(r) - 1
    png = build(r, c, part_log2=10)
    x0 = torch.full((n,), 1.0 / n, dtype=torch.float32, device="cuda")
    y, res = P.iterate(png, x0, d=0.85)
    o = oracle.pagerank(r, c, iters=1)
    assert_ranks_close(y.cpu().numpy(), o.x)
    assert abs(res - o.res_hist[0]) <= 1e-6 * o.res_hist[0] + 1e-9


@pytest.mark.parametrize("relabel", ["random", None])
def test_rmat16_twenty_iterations(relabel):
    """RMAT-16 (65,536 nodes, edge factor 16), 20 fixed iterations, damping
    0.85, dangling mass spread uniformly, FP32 ranks vs the FP64 oracle."""
    r, c = graphgen.rmat(16, 16, seed=1, relabel=relabel)
    png = build(r, c)
    res = P.pagerank(png, d=0.85, tol=0.0, max_iters=20)
    assert res.iters == 20 and res.status == P.PCPM_OK
    o = oracle.pagerank(r, c, d=0.85, iters=20)
    assert_ranks_close(res.pr.cpu().numpy(), o.x)
    np.testing.assert_allclose(res.res_hist, o.res_hist, rtol=0.05, atol=2e-7)
    assert abs(float(res.pr.double().sum()) - 1.0) < 1e-5


@pytest.mark.parametrize("order", [1, 2])
def test_rmat20_multi_workgroup_tile_scans(order):
    """RMAT-20 (16.8M edge draws): over 8192 tiles of destination IDs, so the
    flag prefixes before each tile come from the multi-workgroup scan; exact
    layout and 20 iterations against the oracle, in both update orders."""
    r, c = graphgen.rmat(20, 16, seed=4, relabel="random")
    png = build(r, c, update_order=order)
    assert len(c) > 8192 * 1024 and png.info["update_order"] == order
    assert_layout_equal(png, r, c, 14)
    res = P.pagerank(png, d=0.85, tol=0.0, max_iters=20)
    o = oracle.pagerank(r, c, d=0.85, iters=20)
    assert_ranks_close(res.pr.cpu().numpy(), o.x)
    np.testing.assert_allclose(res.res_hist, o.res_hist, rtol=0.05, atol=2e-7)


@pytest.mark.parametrize("part_log2,sc,gc", [(14, 0, 0), (10, 4096, 4096), (12, 0, 65536), (6, 512, 300)])
def test_to_tolerance_with_split_work(part_log2, sc, gc):
    """Convergence to L1 residual 1e-6; small chunk sizes force split scatter
    partitions and split gather bins (merged in a second pass)."""
    r, c = graphgen.rmat(15, 16, seed=5, relabel="indegree")
    png = build(r, c, part_log2=part_log2, scatter_chunk=sc, gather_chunk=gc)
    if gc:
        assert png.info["split_bins"] > 0
    res = P.pagerank(png, d=0.85, tol=1e-6, max_iters=200)
    assert res.converged and res.resid < 1e-6
    assert np.all(res.res_hist[:-1] >= 1e-6)
    o = oracle.pagerank(r, c, d=0.85, iters=res.iters)
    assert_ranks_close(res.pr.cpu().numpy(), o.x)


def test_init_vector_and_restart():
    """Ten iterations, then ten more from that output, equal twenty in a row
    (checkpoint/resume by passing the rank vector back as init)."""
    r, c = graphgen.rmat(13, 8, seed=9, relabel="random")
    png = build(r, c, part_log2=9)
    a = P.pagerank(png, tol=0.0, max_iters=10)
    b = P.pagerank(png, tol=0.0, max_iters=10, init=a.pr.clone())
    full = P.pagerank(png, tol=0.0, max_iters=20)
    np.testing.assert_allclose(b.pr.cpu().numpy(), full.pr.cpu().numpy(), rtol=1e-5, atol=1e-9)
    o = oracle.pagerank(r, c, iters=20)
    assert_ranks_close(b.pr.cpu().numpy(), o.x)


def test_degenerate_graphs():
    # no edges: every node dangling, ranks stay uniform
    r, c = csr(77, np.zeros((0, 2)))
    res = P.pagerank(build(r, c, part_log2=3), tol=0.0, max_iters=3)
    np.testing.assert_allclose(res.pr.cpu().numpy(), 1 / 77, rtol=1e-6)
    # directed cycle: uniform
    n = 1000
    r, c = csr(n, [(i, (i + 1) % n) for i in range(n)])
    res = P.pagerank(build(r, c, part_log2=5), tol=0.0, max_iters=5)
    np.testing.assert_allclose(res.pr.cpu().numpy(), 1 / n, rtol=1e-6)
    # in-star closed form
    n, d = 5, 0.85
    r, c = csr(n, [(i, 0) for i in range(1, n)])
    res = P.pagerank(build(r, c, part_log2=1), d=d, tol=1e-9, max_iters=500)
    x = res.pr.cpu().numpy()
    assert abs(x[0] - (1 + (n - 1) * d) / (n + (n - 1) * d)) < 1e-6
    # one node
    r, c = csr(1, np.zeros((0, 2)))
    assert P.pagerank(build(r, c), tol=0.0, max_iters=2).pr.item() == pytest.approx(1.0)


# ------------------------------------------------------------------ errors

def test_invalid_graphs_are_rejected():
    good_r, good_c = csr(6, [(0, 1), (0, 2), (1, 2), (3, 4)])
    cases = {
        "unsorted": (good_r, np.array([2, 1, 2, 4], np.int32)),
        "duplicate": (good_r, np.array([1, 1, 2, 4], np.int32)),
        "self_loop": (good_r, np.array([0, 2, 2, 4], np.int32)),
        "out_of_range": (good_r, np.array([1, 2, 2, 6], np.int32)),
        "bad_offsets": (np.array([0, 2, 1, 3, 4, 4, 4], np.int32), good_c),
        "bad_total": (np.array([0, 2, 3, 3, 4, 4, 3], np.int32), good_c),
    }
    for name, (r, c) in cases.items():
        with pytest.raises(P.PCPMError) as ei:
            build(r, c, part_log2=1)
        assert ei.value.status == P.PCPM_ERR_GRAPH, name
    with pytest.raises(P.PCPMError) as ei:
        build(good_r, good_c, part_log2=16)
    assert ei.value.status == P.PCPM_ERR_INVALID_ARG
    png = build(good_r, good_c, part_log2=1)
    with pytest.raises(P.PCPMError) as ei:
        P.pagerank(png, d=1.0)
    assert ei.value.status == P.PCPM_ERR_INVALID_ARG
    with pytest.raises(TypeError):
        P.build_png(torch.from_numpy(good_r), torch.from_numpy(good_c))  # host tensors


def test_not_converged_keeps_valid_output():
    r, c = graphgen.rmat(12, 16, seed=3, relabel="random")
    png = build(r, c, part_log2=8)
    res = P.pagerank(png, tol=1e-12, max_iters=5)
    assert res.status == P.PCPM_ERR_NOT_CONVERGED and res.iters == 5 and not res.converged
    assert_ranks_close(res.pr.cpu().numpy(), oracle.pagerank(r, c, iters=5).x)


@pytest.mark.parametrize("max_iters", [1, 2, 3, 4, 5, 7, 8, 9, 13, 30])
def test_queued_iterations_past_the_end_change_nothing(max_iters):
    """The solve keeps batches of iterations in flight while the host reads
    the control block: whatever it queues past convergence or past max_iters
    must leave the result, the iteration count and the residual history those
    of exactly that many iterations."""
    r, c = graphgen.rmat(12, 16, seed=4, relabel="random")
    png = build(r, c, part_log2=8)
    fixed = P.pagerank(png, tol=0.0, max_iters=max_iters)
    assert fixed.iters == max_iters
    capped = P.pagerank(png, tol=1e-12, max_iters=max_iters)
    assert capped.status == P.PCPM_ERR_NOT_CONVERGED and capped.iters == max_iters
    np.testing.assert_array_equal(capped.pr.cpu().numpy().view(np.uint32), fixed.pr.cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(capped.res_hist, fixed.res_hist)
    # to a tolerance the solve stops after the first iteration below it
    tol = float(fixed.res_hist[-1]) * 1.0000001
    conv = P.pagerank(png, tol=tol, max_iters=100)
    first = int(np.argmax(fixed.res_hist < tol)) + 1
    assert conv.converged and conv.iters == first
    again = P.pagerank(png, tol=0.0, max_iters=first)
    np.testing.assert_array_equal(conv.pr.cpu().numpy().view(np.uint32), again.pr.cpu().numpy().view(np.uint32))


def test_timing_counts_only_the_iterations_that_ran():
    """Per-kernel timing leaves out the launches of iterations queued past
    convergence (they return at once and would dilute the averages): a solve
    of c iterations records c launches of each per-iteration kernel, in PageRank
    and in batched personalised PageRank."""
    r, c = graphgen.rmat(12, 16, seed=4, relabel="random")
    n = len(r) - 1
    png = build(r, c, part_log2=8)
    P.timing_collect()
    P.timing_enable(True)
    try:
        res = P.pagerank(png, tol=1e-6, max_iters=100)
        torch.cuda.synchronize()
        kt = P.timing_collect()
        assert res.converged
        for name in ("pcpm_scatter", "pcpm_gather", "pcpm_finalize"):
            assert kt[name][0] == res.iters, (name, kt[name], res.iters)
        off, seeds = graphgen.seed_sets(n, 3, seed=4)
        ppr = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=100)
        torch.cuda.synchronize()
        kt = P.timing_collect()
        assert ppr.converged
        # three vectors share one tile: the batch runs as long as its slowest vector
        assert kt["pcpm_ppr_gather"][0] == int(ppr.iters.max())
    finally:
        P.timing_enable(False)
        P.timing_collect()


def test_poisoned_init_is_reported():
    r, c = graphgen.rmat(10, 8, seed=3)
    n = len(r) - 1
    png = build(r, c, part_log2=6)
    bad = torch.full((n,), 1.0 / n, device="cuda")
    bad[5] = float("nan")
    with pytest.raises(P.PCPMError) as ei:
        P.pagerank(png, init=bad, tol=1e-6, max_iters=10)
    assert ei.value.status == P.PCPM_ERR_NUMERIC


def test_poisoned_input_without_resid_gives_nan():
    """pcpm_iterate with resid NULL does not synchronise; a non-finite input
    makes the whole output NaN instead of leaving it unwritten."""
    r, c = graphgen.rmat(10, 8, seed=3)
    n = len(r) - 1
    png = build(r, c, part_log2=6)
    bad = torch.full((n,), 1.0 / n, device="cuda")
    bad[7] = float("inf")
    out = torch.zeros(n, device="cuda")
    P.iterate(png, bad, pr_out=out, want_resid=False)
    assert torch.isnan(out).all().item()
    with pytest.raises(P.PCPMError) as ei:
        P.iterate(png, bad, pr_out=out, want_resid=True)
    assert ei.value.status == P.PCPM_ERR_NUMERIC
    # a finite input afterwards is computed normally
    good = torch.full((n,), 1.0 / n, device="cuda")
    y, _ = P.iterate(png, good, pr_out=out, want_resid=False)
    assert_ranks_close(y.cpu().numpy(), oracle.pagerank(r, c, iters=1).x)


@pytest.mark.parametrize("scale", [1e20, 1e30])
def test_start_vector_of_large_values(scale):
    """A start vector of L1 mass far above 2^60 (the fixed-point scale goes
    below one unit) iterates as the oracle does from the same vector, used as
    given."""
    r, c = graphgen.rmat(12, 8, seed=13, relabel="random")
    n = len(r) - 1
    png = build(r, c, part_log2=8)
    rng = np.random.default_rng(5)
    x0 = (rng.random(n) * (2.0 * scale / n)).astype(np.float32)
    assert np.isfinite(x0).all()
    res = P.pagerank(png, tol=0.0, max_iters=4, init=torch.from_numpy(x0).cuda())
    o = oracle.pagerank(r, c, iters=4, x0=x0.astype(np.float64))
    got = res.pr.cpu().numpy().astype(np.float64)
    mass = np.abs(o.x).sum()
    assert np.abs(got - o.x).sum() <= 1e-5 * mass
    big = o.x > mass / n
    assert (np.abs(got - o.x)[big] / o.x[big]).max() <= 1e-3
    np.testing.assert_allclose(res.res_hist, o.res_hist, rtol=1e-4)
