"""GPU parity of pcpm_relabel (degree-ordered labelling, Sec. 5.3.1 / Table 6)
with oracle.relabel: permutation and relabelled CSR bit-exact; errors; and
PageRank on the relabelled graph equal to the original's, moved by perm."""
import ctypes

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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def check_exact(r, c, key):
    perm, ro2, c2 = P.relabel(dev(r), dev(c), key=key)
    want = oracle.relabel(r, c, key=key)
    np.testing.assert_array_equal(perm.cpu().numpy(), want[0])
    np.testing.assert_array_equal(ro2.cpu().numpy(), want[1])
    np.testing.assert_array_equal(c2.cpu().numpy(), want[2])
    return perm, ro2, c2


def csr(n, edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return graphgen.from_edges(n, e[:, 0], e[:, 1], threads=1)


@pytest.mark.parametrize("key", ["in", "out"])
@pytest.mark.parametrize("scale,ef,relabel", [(12, 16, "random"), (14, 8, None), (10, 4, "indegree")])
def test_rmat_exact(scale, ef, relabel, key):
    r, c = graphgen.rmat(scale, ef, seed=scale, relabel=relabel)
    check_exact(r, c, key)


@pytest.mark.parametrize("key", ["in", "out"])
def test_ragged_and_degenerate(key):
    rng = np.random.default_rng(7)
    for n, p in ((1, 0.0), (2, 1.0), (3, 0.5), (77, 0.1), (1500, 0.004)):
        a = rng.random((n, n)) < p
        np.fill_diagonal(a, False)
        u, v = np.nonzero(a)
        r, c = csr(n, np.stack([u, v], 1))
        check_exact(r, c, key)
    # no edges at all
    check_exact(np.zeros(6, np.int32), np.zeros(0, np.int32), key)
    # a star into node 3 and a hub row of 9000 edges (several 1024-edge tiles,
    # long runs of empty rows between)
    n = 20000
    edges = [(u, 3) for u in range(0, n, 7) if u != 3] + [(11, v) for v in range(9001) if v != 11]
    r, c = csr(n, edges)
    check_exact(r, c, key)


def test_rmat20_multi_tile_sorts():
    """16M edges: thousands of 4096-key tiles per pass, multi-workgroup scans."""
    r, c = graphgen.rmat(20, 16, seed=6, relabel="random")
    check_exact(r, c, "in")


def test_relabelled_pagerank_matches():
    r, c = graphgen.rmat(16, 16, seed=8, relabel="random")
    perm, ro2, c2 = P.relabel(dev(r), dev(c), key="in")
    a = P.pagerank(P.build_png(dev(r), dev(c)), d=0.85, tol=0.0, max_iters=20).pr.cpu().numpy()
    png2 = P.build_png(ro2, c2)
    b = P.pagerank(png2, d=0.85, tol=0.0, max_iters=20).pr.cpu().numpy()
    p = perm.cpu().numpy()
    x = oracle.pagerank(r, c, d=0.85, iters=20).x
    assert np.abs(b[p] - x).sum() <= 1e-5 and np.abs(a - x).sum() <= 1e-5
    # in-degree order packs the hubs into few partitions: fewer PNG edges
    assert png2.info["eprime"] < P.build_png(dev(r), dev(c)).info["eprime"]


def test_errors():
    r, c = graphgen.rmat(10, 8, seed=2)
    bad = np.array(c, dtype=np.int32)
    bad[5] = len(r) - 1 + 3  # column outside [0, n)
    with pytest.raises(P.PCPMError) as e:
        P.relabel(dev(r), dev(bad))
    assert e.value.status == P.PCPM_ERR_GRAPH
    ro = np.array(r, dtype=np.int32)
    ro[4] = ro[5] + 1  # decreasing offsets
    with pytest.raises(P.PCPMError) as e:
        P.relabel(dev(ro), dev(c))
    assert e.value.status == P.PCPM_ERR_GRAPH
    with pytest.raises(ValueError):
        P.relabel(dev(r), dev(c), key="pagerank")
    # key outside {0, 1} and overlapping outputs, through the C ABI directly
    rd, cd = dev(r), dev(c)
    n, m = len(r) - 1, len(c)
    out = torch.empty(2 * n + 1 + m, dtype=torch.int32, device="cuda")
    lib = P.lib()
    vp = lambda t, o=0: ctypes.c_void_p(t.data_ptr() + 4 * o)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.pcpm_relabel(n, m, vp(rd), vp(cd), 2, vp(out), vp(out, n), vp(out, 2 * n + 1), st) == P.PCPM_ERR_INVALID_ARG
    assert lib.pcpm_relabel(n, m, vp(rd), vp(cd), 0, vp(out), vp(out, 1), vp(out, 2 * n + 1), st) == P.PCPM_ERR_INVALID_ARG
    assert lib.pcpm_relabel(n, m, vp(rd), vp(cd), 0, vp(out), vp(rd), vp(out, 2 * n + 1), st) == P.PCPM_ERR_INVALID_ARG
    assert lib.pcpm_relabel(n, m, vp(rd), vp(cd), 0, vp(out), vp(out, n), vp(out, 2 * n + 1), st) == P.PCPM_OK
