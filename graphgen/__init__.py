"""Seeded synthetic graph inputs in canonical CSR form.

This module produces inputs only (no PageRank arithmetic).  The CPU oracle and
the GPU library are both fed from it, so the two sides always see the same
graph for the same seed.

Canonical form: self-loops and duplicate edges dropped, rows sorted ascending,
int32 ``row_off[n+1]`` / ``col[m]``, isolated nodes kept.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc/OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    vp, i64, u64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    lib.gg_rmat.restype = vp
    lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, u64, ctypes.c_int]
    lib.gg_uniform.restype = vp
    lib.gg_uniform.argtypes = [i64, i64, u64, ctypes.c_int]
    lib.gg_from_edges.restype = vp
    lib.gg_from_edges.argtypes = [i64, i64, i32p, i32p, ctypes.c_int]
    lib.gg_nodes.restype = i64
    lib.gg_nodes.argtypes = [vp]
    lib.gg_edges.restype = i64
    lib.gg_edges.argtypes = [vp]
    lib.gg_take.restype = ctypes.c_int
    lib.gg_take.argtypes = [vp, i32p, i32p]
    lib.gg_discard.restype = None
    lib.gg_discard.argtypes = [vp]
    lib.gg_perm_random.restype = ctypes.c_int
    lib.gg_perm_random.argtypes = [i64, u64, i32p]
    lib.gg_perm_indegree.restype = ctypes.c_int
    lib.gg_perm_indegree.argtypes = [i64, i32p, i32p, i32p, ctypes.c_int]
    lib.gg_relabel.restype = ctypes.c_int
    lib.gg_relabel.argtypes = [i64, i32p, i32p, i32p, i32p, i32p, ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _take(h) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    if not h:
        raise ValueError("graph generator rejected its arguments")
    n = lib.gg_nodes(h)
    m = lib.gg_edges(h)
    row_off = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(m, 1), dtype=np.int32)[:m]
    if lib.gg_take(h, _ptr(row_off), _ptr(col) if m else _ptr(np.empty(1, np.int32))) != 0:
        raise OverflowError("edge count does not fit int32 offsets")
    return row_off, col


def _threads(threads):
    if threads is not None:
        return int(threads)
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def rmat(scale: int, edge_factor: float = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, relabel: str | None = None, threads: int | None = None):
    """Directed RMAT graph: 2**scale nodes, edge_factor * 2**scale edge draws.

    relabel: None (generator labels), "random" (seeded uniform permutation of
    both endpoints) or "indegree" (in-degree descending, ties by generator ID).
    """
    lib = _load()
    t = _threads(threads)
    h = lib.gg_rmat(int(scale), float(edge_factor), float(a), float(b), float(c),
                    int(seed) & (2**64 - 1), t)
    row_off, col = _take(h)
    if relabel is None:
        return row_off, col
    n = len(row_off) - 1
    newid = np.empty(n, dtype=np.int32)
    if relabel == "random":
        lib.gg_perm_random(n, (int(seed) * 7919 + 17) & (2**64 - 1), _ptr(newid))
    elif relabel == "indegree":
        lib.gg_perm_indegree(n, _ptr(row_off), _ptr(col) if len(col) else _ptr(newid),
                             _ptr(newid), t)
    else:
        raise ValueError(f"unknown relabel {relabel!r}")
    return apply_labels(row_off, col, newid, threads=t)


def apply_labels(row_off: np.ndarray, col: np.ndarray, newid: np.ndarray, threads=None):
    """Relabel node v as newid[v] (a permutation) and re-canonicalise."""
    lib = _load()
    n = len(row_off) - 1
    row_off = np.ascontiguousarray(row_off, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    newid = np.ascontiguousarray(newid, dtype=np.int32)
    r2 = np.empty(n + 1, dtype=np.int32)
    c2 = np.empty(max(len(col), 1), dtype=np.int32)
    dummy = np.empty(1, dtype=np.int32)
    rc = lib.gg_relabel(n, _ptr(row_off), _ptr(col) if len(col) else _ptr(dummy), _ptr(newid),
                        _ptr(r2), _ptr(c2), _threads(threads))
    if rc != 0:
        raise ValueError("newid is not a permutation")
    return r2, c2[: len(col)]


def indegree_labels(row_off, col, threads=None) -> np.ndarray:
    lib = _load()
    n = len(row_off) - 1
    newid = np.empty(n, dtype=np.int32)
    row_off = np.ascontiguousarray(row_off, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    lib.gg_perm_indegree(n, _ptr(row_off), _ptr(col) if len(col) else _ptr(newid), _ptr(newid),
                         _threads(threads))
    return newid


def uniform(n: int, m_draws: int, seed: int = 4, threads: int | None = None):
    """Directed graph with both endpoints of every edge drawn uniformly from [0,n)."""
    lib = _load()
    h = lib.gg_uniform(int(n), int(m_draws), int(seed) & (2**64 - 1), _threads(threads))
    return _take(h)


def from_edges(n: int, src, dst, threads: int | None = None):
    """Canonical CSR of an explicit edge list."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    dummy = np.zeros(1, dtype=np.int32)
    h = lib.gg_from_edges(int(n), len(src), _ptr(src) if len(src) else _ptr(dummy),
                          _ptr(dst) if len(dst) else _ptr(dummy), _threads(threads))
    return _take(h)


def seed_sets(n: int, k: int, seed: int, lo: int = 1, hi: int = 100):
    """k teleport seed sets, |S_j| uniform in [lo, hi], members uniform without
    replacement over [0, n).  Returns (seed_off[k+1], seeds) as int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(lo, min(hi, n) + 1, size=k)
    off = np.zeros(k + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    seeds = np.empty(int(off[-1]), dtype=np.int32)
    for j in range(k):
        s = rng.choice(n, size=int(sizes[j]), replace=False)
        seeds[off[j]:off[j + 1]] = np.sort(s)
    return off.astype(np.int32), seeds


def uneven_rmat_batch(count: int = 16, seed: int = 100, scales=(14, 20), edge_factors=(8, 32),
                      relabel: str | None = "random"):
    """`count` RMAT graphs of uneven size: scale and (integer) edge factor
    drawn uniformly from the given inclusive ranges, graph i seeded seed + i;
    the first graph takes the smallest scale and edge factor, the last the
    largest, so both extremes are present.  Returns ([(row_off, col)], [(scale,
    edge_factor)])."""
    rng = np.random.default_rng(seed)
    sc = rng.integers(scales[0], scales[1] + 1, count)
    ef = rng.integers(edge_factors[0], edge_factors[1] + 1, count)
    sc[0], ef[0], sc[-1], ef[-1] = scales[0], edge_factors[0], scales[1], edge_factors[1]
    graphs = [rmat(int(s), int(e), seed=seed + i, relabel=relabel) for i, (s, e) in enumerate(zip(sc, ef))]
    return graphs, [(int(s), int(e)) for s, e in zip(sc, ef)]
