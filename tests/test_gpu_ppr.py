"""Batched personalised PageRank (pcpm_ppr_batch) against the FP64 oracle,
vector by vector, at the GPU's per-vector iteration count."""
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


def check_vectors(x, r, c, off, seeds, iters, d=0.85):
    n = len(r) - 1
    for j in range(len(off) - 1):
        s = seeds[off[j]:off[j + 1]]
        ref = oracle.ppr(r, c, s, d=d, iters=int(iters[j])).x
        got = x[:, j].astype(np.float64)
        l1 = np.abs(got - ref).sum()
        assert l1 <= 1e-5, (j, l1)
        big = ref > 1.0 / n
        if big.any():
            assert (np.abs(got - ref)[big] / ref[big]).max() <= 1e-3, j


@pytest.mark.parametrize("k,part_log2", [(8, 11), (13, 10), (32, 10), (5, 8), (64, 9)])
def test_ppr_fixed_iterations(k, part_log2):
    r, c = graphgen.rmat(13, 16, seed=4, relabel="random")
    n = len(r) - 1
    png = P.build_png(dev(r), dev(c), part_log2=part_log2)
    off, seeds = graphgen.seed_sets(n, k, seed=k)
    res = P.ppr_batch(png, off, seeds, tol=0.0, max_iters=15)
    assert np.all(res.iters == 15)
    x = res.pr.cpu().numpy()
    check_vectors(x, r, c, off, seeds, res.iters)
    np.testing.assert_allclose(x.sum(axis=0), 1.0, atol=1e-4)


def test_ppr_to_tolerance_with_split_bins():
    r, c = graphgen.rmat(14, 16, seed=6)  # generator labels: hubs share partitions
    n = len(r) - 1
    png = P.build_png(dev(r), dev(c), part_log2=10, gather_chunk=8192, scatter_chunk=4096)
    assert png.info["split_bins"] > 0
    off, seeds = graphgen.seed_sets(n, 24, seed=9)
    res = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=200)
    assert res.converged and np.all(res.resid < 1e-6)
    check_vectors(res.pr.cpu().numpy(), r, c, off, seeds, res.iters)


def test_ppr_on_every_node_is_plain_pagerank():
    r, c = graphgen.rmat(11, 8, seed=3, relabel="random")
    n = len(r) - 1
    png = P.build_png(dev(r), dev(c), part_log2=9)
    off = np.array([0, n], np.int32)
    seeds = np.arange(n, dtype=np.int32)
    a = P.ppr_batch(png, off, seeds, tol=0.0, max_iters=12).pr.cpu().numpy()[:, 0]
    b = P.pagerank(png, tol=0.0, max_iters=12).pr.cpu().numpy()
    np.testing.assert_allclose(a, b, rtol=2e-6, atol=1e-10)


def test_ppr_cycle_closed_form():
    n, d, s = 40, 0.85, 7
    e = np.array([(i, (i + 1) % n) for i in range(n)])
    r, c = graphgen.from_edges(n, e[:, 0], e[:, 1])
    png = P.build_png(dev(r), dev(c), part_log2=3)
    res = P.ppr_batch(png, np.array([0, 1], np.int32), np.array([s], np.int32), d=d, tol=1e-9, max_iters=2000)
    ell = (np.arange(n) - s) % n
    want = (1 - d) * d ** ell / (1 - d ** n)
    assert np.abs(res.pr.cpu().numpy()[:, 0] - want).sum() < 2e-6


def test_ppr_rejects_bad_seed_sets():
    r, c = graphgen.rmat(8, 8, seed=1)
    png = P.build_png(dev(r), dev(c), part_log2=5)
    for off, seeds in [([0, 0], []), ([0, 2], [3, 3]), ([0, 1], [256]), ([0, 1], [-1])]:
        with pytest.raises(P.PCPMError) as ei:
            P.ppr_batch(png, np.array(off, np.int32), np.array(seeds, np.int32))
        assert ei.value.status == P.PCPM_ERR_INVALID_ARG


@pytest.mark.parametrize("k,part_log2", [(37, 12), (37, 10), (21, 11)])
def test_ppr_queue_refill_matches_single_vectors(k, part_log2):
    """More vectors than slots: a slot whose vector converges starts the next
    one.  Every vector matches the oracle at its own iteration count, and that
    count is the one it takes when run alone (up to one iteration where its
    residual sits at tol: the tile's shared fixed-point scale rounds
    differently)."""
    r, c = graphgen.rmat(13, 16, seed=8, relabel="random")
    n = len(r) - 1
    png = P.build_png(dev(r), dev(c), part_log2=part_log2)
    assert P.ppr_tile_width(png) < k
    off, seeds = graphgen.seed_sets(n, k, seed=40 + k)
    res = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=200)
    assert res.converged and np.all(res.resid < 1e-6)
    x = res.pr.cpu().numpy()
    check_vectors(x, r, c, off, seeds, res.iters)
    np.testing.assert_allclose(x.sum(axis=0), 1.0, atol=1e-4)
    alone = np.array([P.ppr_batch(png, off[j:j + 2] - off[j], seeds[off[j]:off[j + 1]], tol=1e-6,
                                  max_iters=200).iters[0] for j in range(k)])
    assert np.all(np.abs(res.iters - alone) <= 1), (res.iters, alone)
    assert np.mean(res.iters == alone) >= 0.9
    png.close()


def test_ppr_queue_mixes_fast_slow_and_capped_vectors():
    """A cycle of 48 nodes plus 48 isolated (dangling) nodes.  A vector seeded
    on isolated nodes is a fixed point after one iteration (all its mass
    teleports back); one seeded on the cycle needs many.  With max_iters = 30
    the cycle vectors stop unconverged while the others finish at once and
    free their slots; all of them are stored at their own counts."""
    nc, ni, d = 48, 48, 0.85
    n = nc + ni
    e = np.array([(i, (i + 1) % nc) for i in range(nc)])
    r, c = graphgen.from_edges(n, e[:, 0], e[:, 1])
    png = P.build_png(dev(r), dev(c), part_log2=3)
    kt = P.ppr_tile_width(png)
    sets = []
    for j in range(3 * kt):
        if j % 4 == 3:
            sets.append([j % nc, (j + 5) % nc])          # on the cycle: slow
        else:
            sets.append([nc + (j % ni), nc + ((j + 7) % ni)])  # isolated: one iteration
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int32)
    seeds = np.concatenate(sets).astype(np.int32)
    res = P.ppr_batch(png, off, seeds, d=d, tol=1e-9, max_iters=30)
    assert not res.converged
    slow = np.array([j % 4 == 3 for j in range(len(sets))])
    assert np.all(res.iters[~slow] == 1) and np.all(res.resid[~slow] < 1e-9)
    assert np.all(res.iters[slow] == 30) and np.all(res.resid[slow] > 1e-9)
    x = res.pr.cpu().numpy()
    check_vectors(x, r, c, off, seeds, res.iters, d=d)
    for j, s in enumerate(sets):
        if not slow[j]:
            want = np.zeros(n)
            want[s] = 0.5
            np.testing.assert_allclose(x[:, j], want, atol=1e-7)
    png.close()
