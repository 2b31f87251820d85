"""The autotuner (pcpm_build_png with part_log2 = 0): the measured sweep of
partition size and update order, then work-item chunks, on the GPU; the
handle it returns has the fastest configuration of its own table, gives
the oracle's ranks, and a second build of the same graph is served from the
process's cache (and, through autotune.tune, from a JSON file)."""
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


def check_vector(got, ref):
    got = np.asarray(got, np.float64)
    assert np.abs(got - ref).sum() <= 1e-5
    big = ref > 1.0 / len(ref)
    assert (np.abs(got - ref)[big] / ref[big]).max() <= 1e-3


def test_part_log2_zero_autotunes_and_caches():
    r, c = graphgen.rmat(14, 16, seed=2, relabel="random")
    rt, ct = dev(r), dev(c)
    P.tune_cache_clear()
    png = P.build_png(rt, ct, part_log2=0, tune_log2_mask=(1 << 8) | (1 << 10) | (1 << 12))
    rows, best, cached = png.tune_table()
    assert not cached
    sweep = [(x["part_log2"], x["update_order"]) for x in rows if x["build_ms"] > 0]
    assert sorted(sweep) == [(p, o) for p in (8, 10, 12) for o in (1, 2)]
    assert len(rows) == 6 + 4  # gather chunk half / double, scatter chunk half / double
    assert rows[best]["ms_per_iter"] == min(x["ms_per_iter"] for x in rows)
    b = rows[best]
    assert png.info["q"] == 1 << b["part_log2"] and png.info["update_order"] == b["update_order"]
    res = P.pagerank(png, tol=0.0, max_iters=20)
    check_vector(res.pr.cpu().numpy(), oracle.pagerank(r, c, iters=20).x)
    # the same graph again: no sweep, the same configuration and table
    again = P.build_png(rt, ct, part_log2=0, tune_log2_mask=(1 << 8) | (1 << 10) | (1 << 12))
    rows2, best2, cached2 = again.tune_table()
    assert cached2 and best2 == best and rows2 == rows
    assert again.info["q"] == png.info["q"] and again.info["gather_items"] == png.info["gather_items"]
    assert torch.equal(P.pagerank(again, tol=0.0, max_iters=20).pr, res.pr)
    # another graph of the same size is tuned afresh (the key holds its content)
    r2, c2 = graphgen.rmat(14, 16, seed=3, relabel="random")
    if len(c2) == len(c):
        other = P.build_png(dev(r2), dev(c2), part_log2=0, tune_log2_mask=(1 << 8) | (1 << 10) | (1 << 12))
        assert not other.tune_table()[2]
    assert P.graph_hash(rt, ct) == P.graph_hash(dev(r), dev(c)) != P.graph_hash(dev(r2), dev(c2))


def test_tune_with_json_cache(tmp_path):
    r, c = graphgen.rmat(13, 16, seed=4, relabel="random")
    rt, ct = dev(r), dev(c)
    cache = str(tmp_path / "tune.json")
    res = P.autotune.tune(rt, ct, candidates=(9, 11), cache=cache, force=True)
    assert res.part_log2 in (9, 11) and not res.cached and res.update_order in (1, 2)
    assert res.ms_per_iter == min(row["ms_per_iter"] for row in res.table)
    again = P.autotune.tune(rt, ct, candidates=(9, 11), cache=cache)
    assert again.cached and (again.part_log2, again.update_order, again.gather_chunk) == (
        res.part_log2, res.update_order, res.gather_chunk)


def test_tune_batched_ppr():
    r, c = graphgen.rmat(13, 16, seed=3, relabel="random")
    n = len(r) - 1
    png, res = P.autotune.build(dev(r), dev(c), vectors=32, candidates=(9, 10, 11, 12))
    assert res.part_log2 in (9, 10, 11, 12)
    assert res.tile_width == min(16, 16384 >> res.part_log2)
    off, seeds = graphgen.seed_sets(n, 8, seed=8)
    out = P.ppr_batch(png, off, seeds, tol=1e-6, max_iters=200)
    assert out.converged
    T = oracle.transpose(r, c)
    for j in range(8):
        check_vector(out.pr.cpu().numpy()[:, j], oracle.ppr(r, c, seeds[off[j]:off[j + 1]], iters=int(out.iters[j]),
                                                            transposed=T).x)


def test_tune_multigraph_union():
    graphs, _ = graphgen.uneven_rmat_batch(6, seed=7, scales=(9, 12), edge_factors=(4, 16))
    r, c, off, sizes = P.union_csr(graphs, 10)
    assert any(o % 2048 for o in off)  # the first graph (512 nodes) is padded to 1024
    png, res = P.autotune.build(dev(r), dev(c), candidates=(9, 10, 11), graph_node_off=off, graph_nodes=sizes)
    assert res.part_log2 in (9, 10)  # 2^11 does not divide the union's offsets: skipped
    assert {row["part_log2"] for row in res.table} == {9, 10}
    out = P.pagerank(png, tol=1e-6, max_iters=200)
    it, _ = png.graph_results()
    x = out.pr.cpu().numpy()
    for g, (rg, cg) in enumerate(graphs):
        check_vector(x[off[g]:off[g] + sizes[g]], oracle.pagerank(rg, cg, iters=int(it[g])).x)
