"""Measured choice of the partition size q and of the update storage order
(and, for batched personalised PageRank, of the vector tile width that q
implies).

The paper picks its partition size by a sweep of execution time against
partition size (Sec. 5.3.2, Figs. 11-14); this does the same sweep on the GPU:
for each candidate q and each update order (bin order, PNG order) it builds
the PNG, runs a few iterations through the library and keeps the fastest time
per iteration (per vector for batched personalised PageRank).  PNG build
time is reported beside it, not mixed in.
Results are cached in a JSON file keyed by (n, m, vectors, device).
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import asdict, dataclass, field

import numpy as np

from . import _pcpm as P

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pcpm_autotune.json")


@dataclass
class TuneResult:
    part_log2: int
    tile_width: int
    ms_per_iter: float           # per vector for batched personalised PageRank
    build_ms: float
    table: list = field(default_factory=list)  # every candidate measured
    cached: bool = False
    update_order: int = 0        # 1 bin order, 2 PNG order (0: entries cached before the order was tuned)


def _device_name():
    import torch

    return torch.cuda.get_device_name(torch.cuda.current_device())


def _key(n, m, vectors):
    return f"n={n};m={m};vectors={vectors};device={_device_name()}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, res: TuneResult):
    db = _load(path)
    d = asdict(res)
    d["cached"] = False
    db[key] = d
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, path)


def _time_solve(fn, iters, reps):
    import torch

    fn(max(1, iters // 2))  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn(iters)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / (reps * iters) * 1e3


def tune(row_off, col, vectors: int = 1, candidates=(12, 13, 14), iters: int = 6, reps: int = 2,
         cache: str | None = DEFAULT_CACHE, seed: int = 0, force: bool = False, orders=(1, 2)) -> TuneResult:
    """Pick part_log2 for PageRank (vectors = 1) or for batched personalised
    PageRank with `vectors` right-hand sides, on device CSR tensors."""
    n, m = row_off.numel() - 1, col.numel()
    key = _key(n, m, vectors)
    if cache and not force:
        hit = _load(cache).get(key)
        if hit:
            hit["cached"] = True
            return TuneResult(**hit)
    rows = []
    cands = [(pl, order) for pl in candidates for order in orders]
    for pl, order in cands:
        if pl < 1 or pl > 14 or (n + (1 << pl) - 1) >> pl > 16384:
            continue
        t0 = time.perf_counter()
        png = P.build_png(row_off, col, part_log2=pl, update_order=order)
        build_ms = (time.perf_counter() - t0) * 1e3
        width = P.ppr_tile_width(png)
        if vectors <= 1:
            ms = _time_solve(lambda it: P.pagerank(png, tol=0.0, max_iters=it, want_hist=False), iters, reps)
            per = ms
        else:
            k = min(vectors, width)
            rng = np.random.default_rng(seed)
            seeds = np.concatenate([np.sort(rng.choice(n, size=min(8, n), replace=False)) for _ in range(k)])
            off = np.arange(0, 8 * k + 1, 8, dtype=np.int32) if n >= 8 else np.arange(0, n * k + 1, n, dtype=np.int32)
            ms = _time_solve(lambda it: P.ppr_batch(png, off, seeds.astype(np.int32), tol=0.0, max_iters=it),
                             iters, reps)
            per = ms / k
        rows.append({"part_log2": pl, "update_order": order, "tile_width": width, "ms_per_iter": per,
                     "build_ms": build_ms, "eprime": png.info["eprime"], "nseg": png.info["nseg"]})
        png.close()
    if not rows:
        raise ValueError("no candidate partition size fits this graph")
    best = min(rows, key=lambda r: r["ms_per_iter"])
    res = TuneResult(best["part_log2"], best["tile_width"], best["ms_per_iter"], best["build_ms"], rows,
                     update_order=best["update_order"])
    if cache:
        _store(cache, key, res)
    return res
