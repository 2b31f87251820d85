"""The partition-size autotuner: measured choice, cached by graph and device."""
import numpy as np
import pytest

import graphgen

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1709_07122_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_tune_pagerank_and_cache(tmp_path):
    r, c = graphgen.rmat(14, 16, seed=2, relabel="random")
    rt, ct = torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()
    cache = str(tmp_path / "tune.json")
    res = P.autotune.tune(rt, ct, candidates=(8, 10, 12), iters=3, reps=1, cache=cache)
    assert res.part_log2 in (8, 10, 12) and not res.cached
    assert len(res.table) == 6 and res.update_order in (1, 2)
    assert {(row["part_log2"], row["update_order"]) for row in res.table} == {(p, o) for p in (8, 10, 12) for o in (1, 2)}
    assert res.ms_per_iter == min(row["ms_per_iter"] for row in res.table)
    again = P.autotune.tune(rt, ct, candidates=(8, 10, 12), cache=cache)
    assert again.cached and again.part_log2 == res.part_log2 and again.update_order == res.update_order


def test_tune_batched_ppr(tmp_path):
    r, c = graphgen.rmat(13, 16, seed=3, relabel="random")
    rt, ct = torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()
    res = P.autotune.tune(rt, ct, vectors=32, candidates=(9, 10, 11, 12), iters=2, reps=1,
                          cache=str(tmp_path / "t.json"))
    assert res.part_log2 in (9, 10, 11, 12)
    assert res.tile_width == min(16, 16384 >> res.part_log2)
