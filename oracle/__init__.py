"""CPU oracle for PCPM PageRank -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it; both sides take their graphs from ``graphgen``.

Everything here is FP64 and follows the paper's definitions directly:

* ``pagerank``   Eq. 1 (Sec. 2.1) in the pull direction of Alg. 1, with the
                 mass of dangling nodes spread by the teleport vector.
* ``ppr``        the same recurrence with a teleport vector uniform on a seed
                 set (personalised PageRank).
* ``png_layout`` the Partition-Node Graph and its bins (Sec. 3.1-3.3) built
                 from the set definitions.
* ``pcpm_iterate`` one iteration carried out over that layout (Alg. 3
                 scatter, Alg. 5 gather, Alg. 2 apply).
* ``step_at``    one step of Eq. 1 from a given vector, at chosen nodes only
                 (for checks on graphs too large for full runs).
* ``spmv``       the sparse matrix-vector product of Sec. 3.5 (weighted
                 graphs): y(v) = sum over edges u->v of w(u,v) x(u).
* ``bin_weights`` edge weights in the order of the destination-ID bins, where
                 Sec. 3.5 stores them.
* ``relabel``    a degree-ordered node labelling and the relabelled CSR
                 (Sec. 5.3.1, Table 6: the compression ratio r, and with it
                 the traffic of Sec. 4, rises with a locality-aware labelling).
* ``mlp``        FP64 reference of the warm-start network (see ``oracle.mlp``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.orc_pagerank.restype = ctypes.c_int
    lib.orc_pagerank.argtypes = [i64, vp, vp, ctypes.c_double, vp, vp, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, vp, vp, vp, vp]
    lib.orc_pagerank_csc.restype = ctypes.c_int
    lib.orc_pagerank_csc.argtypes = [i64, vp, vp, vp, ctypes.c_double, vp, vp, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, vp, vp, vp, vp]
    lib.orc_transpose_into.restype = ctypes.c_int
    lib.orc_transpose_into.argtypes = [i64, vp, vp, vp, vp]
    lib.orc_png_sizes.restype = ctypes.c_int
    lib.orc_png_sizes.argtypes = [i64, vp, vp, i64, vp, vp]
    lib.orc_png_layout.restype = ctypes.c_int
    lib.orc_png_layout.argtypes = [i64, vp, vp, i64, vp, vp, vp, vp, vp, vp]
    lib.orc_step_at.restype = ctypes.c_int
    lib.orc_step_at.argtypes = [i64, vp, vp, ctypes.c_double, vp, vp, vp, i64, ctypes.c_int, vp]
    lib.orc_pcpm_iterate.restype = ctypes.c_int
    lib.orc_pcpm_iterate.argtypes = [i64, vp, i64, vp, vp, vp, vp, vp, vp,
                                     ctypes.c_double, vp, vp, vp, vp]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


_EMPTY_I32 = np.zeros(1, dtype=np.int32)


def _col(col):
    col = np.ascontiguousarray(col, dtype=np.int32)
    return col if len(col) else _EMPTY_I32


def _threads(threads):
    if threads is not None:
        return int(threads)
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


class Result:
    def __init__(self, x, iters, res_hist, converged, sec_per_iter):
        self.x = x
        self.iters = iters
        self.res_hist = res_hist
        self.converged = converged
        self.sec_per_iter = sec_per_iter

    @property
    def resid(self):
        return float(self.res_hist[self.iters - 1]) if self.iters else float("nan")


class Transposed:
    """The transposed adjacency of a CSR graph (in-neighbour lists, sources
    ascending), formed once for many oracle runs on the same graph."""

    def __init__(self, row_off, col):
        lib = _load()
        self.row_off = np.ascontiguousarray(row_off, dtype=np.int32)
        n = len(self.row_off) - 1
        m = int(self.row_off[-1])
        colc = _col(col)
        self.in_off = np.empty(n + 2, dtype=np.int64)
        self.in_src = np.empty(max(m, 1), dtype=np.int32)
        if lib.orc_transpose_into(n, _p(self.row_off), _p(colc), _p(self.in_off), _p(self.in_src)) != 0:
            raise ValueError("oracle rejected its input")


def transpose(row_off, col) -> Transposed:
    return Transposed(row_off, col)


def pagerank(row_off, col, d=0.85, iters=20, tol=0.0, tele=None, x0=None, threads=None,
             transposed: Transposed | None = None) -> Result:
    """FP64 PageRank of Eq. 1.  ``tol > 0`` stops at the first iteration whose
    L1 residual is below ``tol`` (at most ``iters``); otherwise runs exactly
    ``iters`` iterations.  ``transposed`` (from ``transpose(row_off, col)``)
    skips forming the in-neighbour lists again."""
    lib = _load()
    row_off = np.ascontiguousarray(row_off, dtype=np.int32)
    n = len(row_off) - 1
    tele = None if tele is None else np.ascontiguousarray(tele, dtype=np.float64)
    x0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    x = np.empty(n, dtype=np.float64)
    hist = np.zeros(max(iters, 1), dtype=np.float64)
    it = np.zeros(1, dtype=np.int32)
    spi = np.zeros(1, dtype=np.float64)
    if transposed is not None:
        if not np.array_equal(transposed.row_off, row_off):
            raise ValueError("transposed adjacency of another graph")
        rc = lib.orc_pagerank_csc(n, _p(row_off), _p(transposed.in_off), _p(transposed.in_src), float(d),
                                  _p(tele), _p(x0), int(iters), float(tol), _threads(threads), _p(x), _p(hist),
                                  _p(it), _p(spi))
    else:
        colc = _col(col)  # held here: a temporary's buffer could be freed before the call
        rc = lib.orc_pagerank(n, _p(row_off), _p(colc), float(d), _p(tele), _p(x0), int(iters),
                              float(tol), _threads(threads), _p(x), _p(hist), _p(it), _p(spi))
    if rc < 0:
        raise ValueError("oracle rejected its input")
    return Result(x, int(it[0]), hist[: int(it[0])], rc == 0, float(spi[0]))


def step_at(row_off, col, x, nodes, d=0.85, tele=None, threads=None) -> np.ndarray:
    """x_{i+1}(v) of Eq. 1 for v in ``nodes``, from x_i = ``x`` (FP64)."""
    lib = _load()
    row_off = np.ascontiguousarray(row_off, dtype=np.int32)
    n = len(row_off) - 1
    x = np.ascontiguousarray(x, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    tele = None if tele is None else np.ascontiguousarray(tele, dtype=np.float64)
    if len(x) != n:
        raise ValueError("x must have n entries")
    out = np.empty(len(nodes), dtype=np.float64)
    colc = _col(col)  # held here: a temporary's buffer could be freed before the call
    rc = lib.orc_step_at(n, _p(row_off), _p(colc), float(d), _p(tele), _p(x), _p(nodes) if len(nodes) else None,
                         len(nodes), _threads(threads), _p(out))
    if rc < 0:
        raise ValueError("oracle rejected its input")
    return out


def teleport_from_seeds(n, seeds) -> np.ndarray:
    """t(v) = 1/|S| on the seed set S, 0 elsewhere."""
    t = np.zeros(n, dtype=np.float64)
    s = np.unique(np.asarray(seeds, dtype=np.int64))
    t[s] = 1.0 / len(s)
    return t


def ppr(row_off, col, seeds, d=0.85, iters=100, tol=0.0, threads=None,
        transposed: Transposed | None = None) -> Result:
    """Personalised PageRank: the recurrence of Eq. 1 with the uniform jump
    and the dangling redistribution both replaced by t = uniform on ``seeds``;
    starts from x_0 = t."""
    n = len(row_off) - 1
    t = teleport_from_seeds(n, seeds)
    return pagerank(row_off, col, d=d, iters=iters, tol=tol, tele=t, x0=t, threads=threads,
                    transposed=transposed)


class PNG:
    """Canonical PNG arrays (int64 offsets, uint32 destination IDs)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    @property
    def eprime(self):
        return int(self.upd_start[-1])


def png_layout(row_off, col, q: int) -> PNG:
    """Canonical PNG for partitions of ``q`` nodes (any q >= 1)."""
    lib = _load()
    row_off = np.ascontiguousarray(row_off, dtype=np.int32)
    colc = _col(col)
    n = len(row_off) - 1
    m = int(row_off[-1])
    k = np.zeros(1, dtype=np.int64)
    ep = np.zeros(1, dtype=np.int64)
    if lib.orc_png_sizes(n, _p(row_off), _p(colc), int(q), _p(k), _p(ep)) != 0:
        raise ValueError("bad PNG arguments")
    k, ep = int(k[0]), int(ep[0])
    png_off = np.zeros(k * (k + 1), dtype=np.int64)
    png_src = np.zeros(max(ep, 1), dtype=np.int32)
    upd_start = np.zeros(k + 1, dtype=np.int64)
    wo = np.zeros(k * k, dtype=np.int64)
    did_start = np.zeros(k + 1, dtype=np.int64)
    did = np.zeros(max(m, 1), dtype=np.uint32)
    lib.orc_png_layout(n, _p(row_off), _p(colc), int(q), _p(png_off), _p(png_src),
                       _p(upd_start), _p(wo), _p(did_start), _p(did))
    return PNG(n=n, m=m, k=k, q=int(q),
               png_off=png_off.reshape(k, k + 1), png_src=png_src[:ep], upd_start=upd_start,
               wo=wo.reshape(k, k), did_start=did_start, did=did[:m])


def pcpm_iterate(row_off, png: PNG, x, d=0.85, tele=None):
    """One FP64 iteration over the PNG layout (Alg. 3 + Alg. 5 + apply).
    Returns (y, res)."""
    lib = _load()
    row_off = np.ascontiguousarray(row_off, dtype=np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    res = np.zeros(1, dtype=np.float64)
    tele = None if tele is None else np.ascontiguousarray(tele, dtype=np.float64)
    png_src = png.png_src if len(png.png_src) else _EMPTY_I32
    did = png.did if len(png.did) else np.zeros(1, np.uint32)
    lib.orc_pcpm_iterate(png.n, _p(row_off), png.q,
                         _p(np.ascontiguousarray(png.png_off.reshape(-1))), _p(png_src),
                         _p(png.upd_start), _p(np.ascontiguousarray(png.wo.reshape(-1))),
                         _p(png.did_start), _p(did), float(d), _p(tele), _p(x), _p(y), _p(res))
    return y, float(res[0])


def _sources(row_off) -> np.ndarray:
    row_off = np.asarray(row_off, dtype=np.int64)
    return np.repeat(np.arange(len(row_off) - 1, dtype=np.int64), np.diff(row_off))


def spmv(row_off, col, x, weights=None, num_cols=None) -> np.ndarray:
    """Sec. 3.5: y(v) = sum over edges u->v of w(u,v) * x(u) in FP64, with
    w = 1 on every edge when ``weights`` is None (weights[e] belongs to the
    CSR edge row -> col[e]); that is y = A^T x for the CSR matrix A, whose
    columns number ``num_cols`` (the rows' count when None; a non-square A
    gives y a length other than x's)."""
    n = len(row_off) - 1
    x = np.asarray(x, dtype=np.float64)
    col = np.asarray(col, dtype=np.int64)
    w = np.ones(len(col)) if weights is None else np.asarray(weights, dtype=np.float64)
    cols = n if num_cols is None else int(num_cols)
    return np.bincount(col, weights=w * x[_sources(row_off)], minlength=cols).astype(np.float64)[:cols]


def bin_weights(row_off, col, weights, q: int) -> np.ndarray:
    """Sec. 3.5: each weight is stored next to its destination ID, so the
    weights follow the canonical order of the destination-ID bins:
    destination partition, then source partition, source node, destination
    node (the order of ``png_layout(...).did``)."""
    src = _sources(row_off)
    col = np.asarray(col, dtype=np.int64)
    order = np.lexsort((col, src, src // q, col // q))
    return np.asarray(weights)[order]


def relabel(row_off, col, key: str = "in"):
    """Degree-ordered relabelling (Sec. 5.3.1, Table 6: a labelling that puts
    related nodes close raises r).  New label i goes to the node of i-th
    largest in-degree (``key="in"``) or out-degree (``key="out"``), equal
    degrees in increasing old ID.  Returns (perm, row_off2, col2): perm[old]
    = new label; the relabelled CSR holds edge perm[u] -> perm[v] for every
    edge u -> v, rows in ascending column order."""
    row_off = np.asarray(row_off, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(row_off) - 1
    if key == "in":
        deg = np.bincount(col, minlength=n)
    elif key == "out":
        deg = np.diff(row_off)
    else:
        raise ValueError(f"unknown key {key!r}")
    order = np.lexsort((np.arange(n), -deg))  # largest degree first, then old ID
    perm = np.empty(n, dtype=np.int64)
    perm[order] = np.arange(n)
    nu = perm[_sources(row_off)]
    nv = perm[col]
    idx = np.lexsort((nv, nu))
    row_off2 = np.zeros(n + 1, dtype=np.int64)
    row_off2[1:] = np.cumsum(np.bincount(nu, minlength=n))
    return perm, row_off2, nv[idx]
