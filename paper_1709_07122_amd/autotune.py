"""Measured choice of the partition size q, the update storage order and the
work-item chunks (and, for batched personalised PageRank, of the vector tile
width that q implies).

The paper picks its partition size by a sweep of execution time against
partition size (Sec. 5.3.2, Figs. 11-14).  The library runs that sweep
itself when a PNG is built with part_log2 = 0: every candidate q and update
order is built and timed over a few iterations, then the work-item chunks
of the fastest are varied, and the winner is remembered for the process
(keyed by the graph's content hash, the options and the device).  This
module asks for such a build and returns its measurements; it can also keep
the winners in a JSON file across processes, keyed the same way.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass, field

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
    scatter_chunk: int = 0       # work-item chunks of the winner (0: automatic)
    gather_chunk: int = 0


def _device_name():
    import torch

    return torch.cuda.get_device_name(torch.cuda.current_device())


def _mask(candidates) -> int:
    mask = 0
    for pl in candidates:
        if not 1 <= int(pl) <= 14:
            raise ValueError(f"candidate part_log2 {pl} outside [1, 14]")
        mask |= 1 << int(pl)
    return mask


def _key(n, m, content_hash, vectors, mask, graph_node_off=None):
    goff = "" if graph_node_off is None else ",".join(str(int(v)) for v in graph_node_off)
    return (f"n={n};m={m};hash={content_hash:016x};vectors={vectors};mask={mask:x};graphs={goff};"
            f"device={_device_name()}")


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


def result_of(png: P.PNG) -> TuneResult:
    """The TuneResult of an autotuned handle (built with part_log2 = 0)."""
    rows, best, cached = png.tune_table()
    if not rows:
        raise ValueError("the handle was not autotuned (built with a given part_log2)")
    b = rows[best]
    # the PNG build of the winner's q and order (chunk variants reuse it)
    build_ms = next(r["build_ms"] for r in rows
                    if (r["part_log2"], r["update_order"]) == (b["part_log2"], b["update_order"]) and r["build_ms"] > 0)
    return TuneResult(b["part_log2"], P.ppr_tile_width(png), b["ms_per_iter"], build_ms, rows, cached,
                      b["update_order"], b["scatter_chunk"], b["gather_chunk"])


def build(row_off, col, vectors: int = 1, candidates=(12, 13, 14), graph_node_off=None, graph_nodes=None,
          **kw) -> tuple[P.PNG, TuneResult]:
    """An autotuned PNG (the library's sweep) and its TuneResult."""
    png = P.build_png(row_off, col, part_log2=0, tune_vectors=int(vectors), tune_log2_mask=_mask(candidates),
                      graph_node_off=graph_node_off, graph_nodes=graph_nodes, **kw)
    return png, result_of(png)


def tune(row_off, col, vectors: int = 1, candidates=(12, 13, 14), cache: str | None = DEFAULT_CACHE,
         force: bool = False, graph_node_off=None, graph_nodes=None) -> TuneResult:
    """The measured configuration for PageRank (vectors = 1) or for batched
    personalised PageRank with `vectors` right-hand sides, on device CSR
    tensors (a multi-graph union with its graph_node_off / graph_nodes).
    With `cache`, winners are also kept in that JSON file, keyed by the
    graph's content hash, the candidates, the batch and the device."""
    n, m = row_off.numel() - 1, col.numel()
    key = None
    if cache and not force:
        key = _key(n, m, P.graph_hash(row_off, col), vectors, _mask(candidates), graph_node_off)
        hit = _load(cache).get(key)
        if hit:
            hit["cached"] = True
            return TuneResult(**hit)
    if force:
        P.tune_cache_clear()
    png, res = build(row_off, col, vectors, candidates, graph_node_off, graph_nodes)
    png.close()
    if cache:
        key = key or _key(n, m, P.graph_hash(row_off, col), vectors, _mask(candidates), graph_node_off)
        _store(cache, key, res)
    return res
