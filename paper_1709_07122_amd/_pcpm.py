"""ctypes binding of libpcpm (include/pcpm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libpcpm.  PyTorch supplies device memory and the stream.  There is
no CPU fallback; if the library is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcpm.so")

PCPM_OK = 0
PCPM_ERR_INVALID_ARG = 1
PCPM_ERR_GRAPH = 2
PCPM_ERR_OVERFLOW = 3
PCPM_ERR_OOM = 4
PCPM_ERR_DEVICE = 5
PCPM_ERR_NOT_CONVERGED = 6
PCPM_ERR_NUMERIC = 7

STATUS_NAMES = {
    0: "PCPM_OK", 1: "PCPM_ERR_INVALID_ARG", 2: "PCPM_ERR_GRAPH", 3: "PCPM_ERR_OVERFLOW",
    4: "PCPM_ERR_OOM", 5: "PCPM_ERR_DEVICE", 6: "PCPM_ERR_NOT_CONVERGED", 7: "PCPM_ERR_NUMERIC",
}

# every symbol include/pcpm.h declares
EXPORTS = ["pcpm_build_png", "pcpm_png_info", "pcpm_png_export", "pcpm_png_free", "pcpm_iterate",
           "pcpm_pagerank", "pcpm_ppr_batch", "pcpm_ppr_tile_width", "pcpm_graph_results", "pcpm_set_launch", "pcpm_launch_grid", "pcpm_tune_table",
           "pcpm_tune_cache_clear", "pcpm_graph_hash", "pcpm_hbm_stream", "pcpm_last_error",
           "pcpm_timing_enable", "pcpm_timing_collect", "pcpm_ws_features", "pcpm_ws_forward", "pcpm_ws_predict", "pcpm_ws_init",
           "pcpm_ws_work_floats", "pcpm_ws_backward", "pcpm_ws_backward_noalloc", "pcpm_ws_adam", "pcpm_ws_targets", "pcpm_spmv",
           "pcpm_png_export_weights", "pcpm_relabel"]

WS_FEATURES = 8
WS_HIDDEN = 64
WS_PARAMS = 4801


class PCPMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class BuildOpts(ctypes.Structure):
    _fields_ = [("part_log2", ctypes.c_int32), ("num_graphs", ctypes.c_int32),
                ("graph_node_off", ctypes.c_void_p), ("graph_nodes", ctypes.c_void_p),
                ("scatter_chunk", ctypes.c_int64), ("gather_chunk", ctypes.c_int64),
                ("build_chunk", ctypes.c_int64), ("weights", ctypes.c_void_p), ("update_order", ctypes.c_int64),
                ("tune_vectors", ctypes.c_int64), ("tune_log2_mask", ctypes.c_int64),
                ("num_cols", ctypes.c_int64), ("allow_diagonal", ctypes.c_int64)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("part_log2", ctypes.c_int32), ("update_order", ctypes.c_int32),
                ("scatter_chunk", ctypes.c_int64), ("gather_chunk", ctypes.c_int64),
                ("ms_per_iter", ctypes.c_double), ("build_ms", ctypes.c_double)]


class PngInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ("n", "m", "q", "k", "eprime", "nseg", "n_dangling", "scatter_items", "gather_items",
                 "split_bins", "device_bytes", "num_graphs")] + [("build_ms", ctypes.c_double),
                                                                 ("weighted", ctypes.c_int64),
                                                                 ("update_order", ctypes.c_int64),
                                                                 ("num_cols", ctypes.c_int64),
                                                                 ("matrix", ctypes.c_int64)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libpcpm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.pcpm_build_png.restype = ctypes.c_int
    L.pcpm_build_png.argtypes = [i64, i64, vp, vp, ctypes.POINTER(BuildOpts), vp, ctypes.POINTER(vp)]
    L.pcpm_png_info.restype = ctypes.c_int
    L.pcpm_png_info.argtypes = [vp, ctypes.POINTER(PngInfo)]
    L.pcpm_png_export.restype = ctypes.c_int
    L.pcpm_png_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pcpm_png_free.restype = None
    L.pcpm_png_free.argtypes = [vp]
    L.pcpm_png_export_weights.restype = ctypes.c_int
    L.pcpm_png_export_weights.argtypes = [vp, vp]
    L.pcpm_spmv.restype = ctypes.c_int
    L.pcpm_spmv.argtypes = [vp, vp, vp, vp]
    L.pcpm_relabel.restype = ctypes.c_int
    L.pcpm_relabel.argtypes = [i64, i64, vp, vp, i32, vp, vp, vp, vp]
    L.pcpm_iterate.restype = ctypes.c_int
    L.pcpm_iterate.argtypes = [vp, dbl, vp, vp, ctypes.POINTER(dbl), vp]
    L.pcpm_pagerank.restype = ctypes.c_int
    L.pcpm_pagerank.argtypes = [vp, dbl, dbl, i32, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, vp]
    L.pcpm_ppr_batch.restype = ctypes.c_int
    L.pcpm_ppr_batch.argtypes = [vp, dbl, i32, vp, vp, dbl, i32, vp, vp, vp, vp]
    L.pcpm_ppr_tile_width.restype = ctypes.c_int32
    L.pcpm_ppr_tile_width.argtypes = [vp]
    L.pcpm_ws_features.restype = ctypes.c_int
    L.pcpm_ws_features.argtypes = [vp, dbl, vp, ctypes.POINTER(dbl), vp]
    L.pcpm_ws_forward.restype = ctypes.c_int
    L.pcpm_ws_forward.argtypes = [vp, vp, i64, vp, vp]
    L.pcpm_ws_predict.restype = ctypes.c_int
    L.pcpm_ws_predict.argtypes = [vp, vp, dbl, vp, ctypes.POINTER(dbl), vp]
    L.pcpm_ws_init.restype = ctypes.c_int
    L.pcpm_ws_init.argtypes = [vp, i64, vp, vp, ctypes.POINTER(i32), vp]
    L.pcpm_ws_work_floats.restype = i64
    L.pcpm_ws_work_floats.argtypes = [i64]
    L.pcpm_ws_backward.restype = ctypes.c_int
    L.pcpm_ws_backward.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp, ctypes.POINTER(dbl), vp]
    L.pcpm_ws_backward_noalloc.restype = ctypes.c_int
    L.pcpm_ws_backward_noalloc.argtypes = [vp, vp, vp, i64, vp, i64, vp, ctypes.POINTER(dbl), vp]
    L.pcpm_ws_adam.restype = ctypes.c_int
    L.pcpm_ws_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp]
    L.pcpm_ws_targets.restype = ctypes.c_int
    L.pcpm_ws_targets.argtypes = [vp, i64, vp, vp]
    L.pcpm_graph_results.restype = ctypes.c_int
    L.pcpm_graph_results.argtypes = [vp, vp, vp]
    L.pcpm_tune_table.restype = i32
    L.pcpm_tune_table.argtypes = [vp, ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.pcpm_tune_cache_clear.restype = None
    L.pcpm_tune_cache_clear.argtypes = []
    L.pcpm_graph_hash.restype = ctypes.c_int
    L.pcpm_graph_hash.argtypes = [i64, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    L.pcpm_hbm_stream.restype = ctypes.c_int
    L.pcpm_hbm_stream.argtypes = [i32, vp, vp, i64, vp]
    L.pcpm_set_launch.restype = ctypes.c_int
    L.pcpm_set_launch.argtypes = [vp, i32, ctypes.c_uint32]
    L.pcpm_launch_grid.restype = i32
    L.pcpm_launch_grid.argtypes = [vp]
    L.pcpm_last_error.restype = ctypes.c_char_p
    L.pcpm_last_error.argtypes = []
    L.pcpm_timing_enable.restype = None
    L.pcpm_timing_enable.argtypes = [ctypes.c_int]
    L.pcpm_timing_collect.restype = ctypes.c_int
    L.pcpm_timing_collect.argtypes = [ctypes.POINTER(KernelTime), ctypes.c_int]
    _lib = L
    return L


def last_error() -> str:
    return lib().pcpm_last_error().decode()


def _check(status: int, allow=()):
    if status != PCPM_OK and status not in allow:
        raise PCPMError(status, last_error())
    return status


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_tensor(t, dtype, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class PNG:
    """A built Partition-Node Graph (owns device memory in libpcpm)."""

    def __init__(self, handle, row_off, col):
        self._h = handle
        # keep the CSR alive as long as the handle (the handle does not read it
        # after the build, but callers expect the pair to travel together)
        self.row_off = row_off
        self.col = col
        self.info = self._info()

    def _info(self):
        inf = PngInfo()
        _check(lib().pcpm_png_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in PngInfo._fields_}

    @property
    def n(self):
        return self.info["n"]

    @property
    def m(self):
        return self.info["m"]

    @property
    def handle(self):
        if not self._h:
            raise ValueError("PNG handle is closed")
        return self._h

    def export(self) -> dict:
        """Canonical layout as host numpy arrays (see pcpm_png_export)."""
        k, ep, m = self.info["k"], self.info["eprime"], self.info["m"]
        out = dict(png_off=np.zeros(k * (k + 1), np.int64), png_src=np.zeros(max(ep, 1), np.int32),
                   upd_start=np.zeros(k + 1, np.int64), wo=np.zeros(k * k, np.int64),
                   did_start=np.zeros(k + 1, np.int64), did=np.zeros(max(m, 1), np.uint32))
        _check(lib().pcpm_png_export(self.handle, *(ctypes.c_void_p(a.ctypes.data) for a in out.values())))
        out["png_off"] = out["png_off"].reshape(k, k + 1)
        out["wo"] = out["wo"].reshape(k, k)
        out["png_src"] = out["png_src"][:ep]
        out["did"] = out["did"][:m]
        return out

    def export_weights(self) -> np.ndarray:
        """Edge weights in destination-ID bin order (see pcpm_png_export_weights)."""
        w = np.zeros(max(self.m, 1), np.float32)
        _check(lib().pcpm_png_export_weights(self.handle, w.ctypes.data))
        return w[:self.m]

    def graph_results(self):
        """(iters[G], resid[G]) of the last pagerank call on this handle."""
        G = self.info["num_graphs"]
        it = np.zeros(G, np.int32)
        r = np.zeros(G, np.float64)
        _check(lib().pcpm_graph_results(self.handle, it.ctypes.data, r.ctypes.data))
        return it, r

    def tune_table(self):
        """(entries, best index, cached) of an autotuned build (part_log2 = 0);
        entries are dicts of part_log2, update_order, scatter_chunk,
        gather_chunk, ms_per_iter, build_ms."""
        cnt = int(lib().pcpm_tune_table(self.handle, None, 0, None, None))
        arr = (TuneEntry * max(cnt, 1))()
        best, cached = ctypes.c_int32(-1), ctypes.c_int32(0)
        lib().pcpm_tune_table(self.handle, arr, cnt, ctypes.byref(best), ctypes.byref(cached))
        rows = [{f: getattr(arr[i], f) for f, _ in TuneEntry._fields_} for i in range(cnt)]
        return rows, int(best.value), bool(cached.value)

    def set_launch(self, mode: int, spin_limit: int = 0):
        """pcpm_set_launch: 0 automatic, 1 one launch per phase, 2 one
        persistent launch per solve; spin_limit bounds its device-side waits
        (0: the default)."""
        _check(lib().pcpm_set_launch(self.handle, int(mode), int(spin_limit)))

    @property
    def launch_grid(self) -> int:
        """Workgroups of the persistent solve (0: not available)."""
        return int(lib().pcpm_launch_grid(self.handle))

    def close(self):
        if self._h:
            lib().pcpm_png_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_png(row_off, col, part_log2: int = 14, scatter_chunk: int = 0, gather_chunk: int = 0,
              graph_node_off=None, graph_nodes=None, build_chunk: int = 0, weights=None, update_order: int = 0,
              tune_vectors: int = 0, tune_log2_mask: int = 0, num_cols: int = 0, allow_diagonal: int = 0,
              stream=None) -> PNG:
    """pcpm_build_png on device CSR tensors (int32 row_off[n+1], col[m]).

    part_log2 = 0 autotunes (tune_vectors, tune_log2_mask: see
    pcpm_build_opts_t; PNG.tune_table() gives the measurements).
    For several graphs in one handle pass the padded union (see union_csr)
    with its graph_node_off (G+1) and graph_nodes (G).  weights: optional
    device float32 tensor of m edge weights in CSR order (for spmv).
    update_order: 0 automatic, 1 bin order, 2 PNG order (see pcpm_build_opts_t).
    num_cols / allow_diagonal: an n x num_cols matrix (diagonal entries
    allowed) for generic SpMV; such a handle takes spmv only."""
    import torch
    n = row_off.numel() - 1
    m = col.numel()
    rp = _dev_tensor(row_off, torch.int32, name="row_off")
    cp = _dev_tensor(col, torch.int32, name="col") if m else ctypes.c_void_p(0)
    G = 0 if graph_node_off is None else len(graph_nodes)
    goff = np.ascontiguousarray(graph_node_off if G else [0], dtype=np.int64)
    gn = np.ascontiguousarray(graph_nodes if G else [0], dtype=np.int64)
    wp = None if weights is None else _dev_tensor(weights, torch.float32, m, "weights")
    opts = BuildOpts(int(part_log2), G, goff.ctypes.data if G else None, gn.ctypes.data if G else None,
                     int(scatter_chunk), int(gather_chunk), int(build_chunk), wp, int(update_order),
                     int(tune_vectors), int(tune_log2_mask), int(num_cols), int(allow_diagonal))
    h = ctypes.c_void_p()
    _check(lib().pcpm_build_png(n, m, rp, cp, ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
    return PNG(h, row_off, col)


def graph_hash(row_off, col, stream=None) -> int:
    """pcpm_graph_hash: the 64-bit content hash the autotuner's cache keys on."""
    import torch
    n = row_off.numel() - 1
    m = col.numel()
    rp = _dev_tensor(row_off, torch.int32, n + 1, "row_off")
    cp = _dev_tensor(col, torch.int32, m, "col") if m else ctypes.c_void_p(0)
    h = ctypes.c_uint64(0)
    _check(lib().pcpm_graph_hash(n, m, rp, cp, _stream(stream), ctypes.byref(h)))
    return int(h.value)


STREAM_KINDS = {"read": 0, "write": 1, "write_nt": 2, "copy": 3, "copy_nt": 4}


def hbm_stream(kind: str, src, dst, nbytes: int, stream=None):
    """pcpm_hbm_stream: a plain read / write / copy of nbytes on device
    buffers (see the header); asynchronous."""
    import torch
    sp = _dev_tensor(src, torch.float32, name="src") if src is not None else ctypes.c_void_p(0)
    dp = _dev_tensor(dst, torch.float32, name="dst")
    need_dst = 4 * 4096 if kind == "read" else nbytes
    if (src is not None and src.numel() * 4 < nbytes) or dst.numel() * 4 < need_dst:
        raise ValueError("buffers smaller than the stream")
    _check(lib().pcpm_hbm_stream(STREAM_KINDS[kind], sp, dp, int(nbytes), _stream(stream)))


def tune_cache_clear():
    lib().pcpm_tune_cache_clear()


def spmv(png: PNG, x, out=None, stream=None):
    """pcpm_spmv: y(v) = sum over edges u->v of w(u,v) x(u) (w = 1 when the
    handle is unweighted); x (rows) and the returned y (columns) are device
    float32 vectors: both of n entries for a graph."""
    import torch
    n = png.n
    nc = png.info["num_cols"]
    xp = _dev_tensor(x, torch.float32, n, "x")
    if out is None:
        out = torch.empty(nc, dtype=torch.float32, device=x.device)
    yp = _dev_tensor(out, torch.float32, nc, "out")
    _check(lib().pcpm_spmv(png.handle, xp, yp, _stream(stream)))
    return out


RELABEL_KEYS = {"in": 0, "out": 1}


def relabel(row_off, col, key: str = "in", stream=None):
    """pcpm_relabel: degree-ordered labelling (largest in- or out-degree
    first, ties by old ID).  row_off (n+1) and col (m) are device int32
    tensors; returns device int32 tensors (perm, row_off_out, col_out) with
    perm[old] = new label and the relabelled CSR."""
    import torch
    if key not in RELABEL_KEYS:
        raise ValueError(f"key must be one of {sorted(RELABEL_KEYS)}")
    n = row_off.numel() - 1
    m = col.numel()
    rp = _dev_tensor(row_off, torch.int32, n + 1, "row_off")
    cp = _dev_tensor(col, torch.int32, m, "col") if m else ctypes.c_void_p(None)
    perm = torch.empty(n, dtype=torch.int32, device=row_off.device)
    ro2 = torch.empty(n + 1, dtype=torch.int32, device=row_off.device)
    c2 = torch.empty(max(m, 1), dtype=torch.int32, device=row_off.device)[:m]
    _check(lib().pcpm_relabel(n, m, rp, cp, RELABEL_KEYS[key], ctypes.c_void_p(perm.data_ptr()),
                              ctypes.c_void_p(ro2.data_ptr()),
                              ctypes.c_void_p(c2.data_ptr()) if m else ctypes.c_void_p(None), _stream(stream)))
    return perm, ro2, c2


def square_csr(row_off, col, cols: int):
    """A rows x cols CSR matrix as the CSR of a square graph on
    n = max(rows, cols) nodes (rows past `rows` are empty), so that spmv runs
    it: pad x with zeros to n and read y[:cols].  Host arrays in and out; only
    offsets are appended."""
    row_off = np.ascontiguousarray(row_off, dtype=np.int32)
    rows = len(row_off) - 1
    n = max(rows, int(cols))
    if n > rows:
        row_off = np.concatenate([row_off, np.full(n - rows, row_off[-1], np.int32)])
    return row_off, np.ascontiguousarray(col, dtype=np.int32)


def iterate(png: PNG, pr_in, pr_out=None, d: float = 0.85, want_resid: bool = True, stream=None):
    """One PCPM iteration; returns (pr_out, residual or None)."""
    import torch
    n = png.n
    ip = _dev_tensor(pr_in, torch.float32, n, "pr_in")
    if pr_out is None:
        pr_out = torch.empty_like(pr_in)
    op = _dev_tensor(pr_out, torch.float32, n, "pr_out")
    r = ctypes.c_double(0.0)
    _check(lib().pcpm_iterate(png.handle, float(d), ip, op, ctypes.byref(r) if want_resid else None,
                              _stream(stream)))
    return pr_out, (r.value if want_resid else None)


@dataclass
class PagerankResult:
    pr: object
    iters: int
    resid: float
    res_hist: np.ndarray
    converged: bool
    status: int


def pagerank(png: PNG, d: float = 0.85, tol: float = 1e-6, max_iters: int = 100, init=None, out=None,
             want_hist: bool = True, stream=None) -> PagerankResult:
    """pcpm_pagerank: iterate to L1 residual < tol (tol <= 0: exactly max_iters)."""
    import torch
    n = png.n
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=png.row_off.device)
    op = _dev_tensor(out, torch.float32, n, "out")
    ip = _dev_tensor(init, torch.float32, n, "init") if init is not None else None
    it = ctypes.c_int32(0)
    r = ctypes.c_double(0.0)
    hist = np.zeros(max_iters, np.float64)
    st = _check(lib().pcpm_pagerank(png.handle, float(d), float(tol), int(max_iters), ip, op, ctypes.byref(it),
                                    ctypes.byref(r), ctypes.c_void_p(hist.ctypes.data) if want_hist else None,
                                    _stream(stream)), allow=(PCPM_ERR_NOT_CONVERGED,))
    return PagerankResult(out, it.value, r.value, hist[: it.value], st == PCPM_OK and tol > 0, st)


@dataclass
class PprResult:
    pr: object          # [n][k] float32 device tensor
    iters: np.ndarray   # per vector
    resid: np.ndarray   # per vector
    converged: bool
    status: int


def ppr_batch(png: PNG, seed_off, seeds, d: float = 0.85, tol: float = 1e-6, max_iters: int = 100, out=None,
              stream=None) -> PprResult:
    """pcpm_ppr_batch: k personalised PageRank vectors; seed set j is
    seeds[seed_off[j]:seed_off[j+1]] (host int32 arrays)."""
    import torch
    seed_off = np.ascontiguousarray(seed_off, dtype=np.int32)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    k = len(seed_off) - 1
    n = png.n
    if out is None:
        out = torch.empty((n, k), dtype=torch.float32, device=png.row_off.device)
    op = _dev_tensor(out, torch.float32, n * k, "out")
    it = np.zeros(k, np.int32)
    r = np.zeros(k, np.float64)
    st = _check(lib().pcpm_ppr_batch(png.handle, float(d), k, seed_off.ctypes.data,
                                     seeds.ctypes.data if len(seeds) else None, float(tol), int(max_iters), op,
                                     it.ctypes.data, r.ctypes.data, _stream(stream)),
                allow=(PCPM_ERR_NOT_CONVERGED,))
    return PprResult(out, it, r, st == PCPM_OK and tol > 0, st)


def ppr_tile_width(png: PNG) -> int:
    return int(lib().pcpm_ppr_tile_width(png.handle))


def timing_enable(on: bool = True):
    lib().pcpm_timing_enable(1 if on else 0)


def timing_collect() -> dict:
    """{kernel name: (launches, total_ms)} since the last collect."""
    arr = (KernelTime * 64)()
    cnt = lib().pcpm_timing_collect(arr, 64)
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(cnt, 64))}


def union_csr(graphs, part_log2: int):
    """Block-diagonal union of CSR graphs [(row_off, col), ...] in which graph g
    starts at a multiple of q = 2^part_log2 (padding nodes without edges fill
    the gaps).  Returns (row_off, col, graph_node_off[G+1], graph_nodes[G]) as
    host arrays; only IDs are shifted, nothing is computed."""
    q = 1 << part_log2
    offs, sizes, rows, cols = [0], [], [], []
    base_e = 0
    for r, c in graphs:
        r = np.asarray(r, dtype=np.int64)
        n_g = len(r) - 1
        padded = -(-n_g // q) * q
        start = offs[-1]
        rr = np.empty(padded, dtype=np.int64)
        rr[:n_g] = r[:-1] + base_e
        rr[n_g:] = r[-1] + base_e
        rows.append(rr)
        cols.append(np.asarray(c, dtype=np.int64) + start)
        base_e += int(r[-1])
        sizes.append(n_g)
        offs.append(start + padded)
    row_off = np.concatenate(rows + [np.array([base_e])]).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    return row_off, col, np.array(offs, dtype=np.int64), np.array(sizes, dtype=np.int64)


# ---- learned warm start -------------------------------------------------------

def ws_features(png: PNG, d: float = 0.85, stream=None):
    """[n][8] float32 features of every node (pcpm_ws_features); returns
    (features, ms of the per-handle in-degree count done by the first call)."""
    import torch
    feat = torch.empty((png.n, WS_FEATURES), dtype=torch.float32, device=png.row_off.device)
    ms = ctypes.c_double(0.0)
    _check(lib().pcpm_ws_features(png.handle, float(d), _dev_tensor(feat, torch.float32, name="feat"),
                                  ctypes.byref(ms), _stream(stream)))
    return feat, ms.value


def ws_predict(png: PNG, params, d: float = 0.85, out=None, stream=None):
    """The network's prediction for every node of the handle with the
    features formed inside the forward (pcpm_ws_predict): equal to
    ws_forward(params, ws_features(png, d)[0]).  Returns (yhat, ms of the
    per-handle in-degree count done by the first call)."""
    import torch
    if out is None:
        out = torch.empty(png.n, dtype=torch.float32, device=png.row_off.device)
    ms = ctypes.c_double(0.0)
    _check(lib().pcpm_ws_predict(png.handle, _dev_tensor(params, torch.float32, WS_PARAMS, "params"), float(d),
                                 _dev_tensor(out, torch.float32, png.n, "yhat"), ctypes.byref(ms), _stream(stream)))
    return out, ms.value


def ws_forward(params, feat, stream=None):
    import torch
    n = feat.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=feat.device)
    _check(lib().pcpm_ws_forward(_dev_tensor(params, torch.float32, WS_PARAMS, "params"),
                                 _dev_tensor(feat, torch.float32, n * WS_FEATURES, "feat"), n,
                                 _dev_tensor(y, torch.float32, n, "yhat"), _stream(stream)))
    return y


def ws_init(yhat, out=None, stream=None):
    """Softmax of the prediction over the nodes; returns (pr0, used_uniform)."""
    import torch
    n = yhat.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=yhat.device)
    work = torch.empty(int(lib().pcpm_ws_work_floats(1)), dtype=torch.float32, device=yhat.device)
    flag = ctypes.c_int32(0)
    _check(lib().pcpm_ws_init(_dev_tensor(yhat, torch.float32, n, "yhat"), n, _dev_tensor(out, torch.float32, n, "pr0"),
                              _dev_tensor(work, torch.float32, name="work"), ctypes.byref(flag), _stream(stream)))
    return out, bool(flag.value)


def ws_backward(params, feat, target, idx, grad=None, work=None, stream=None):
    """Gradient of the minibatch MSE; returns (grad, loss)."""
    import torch
    b = idx.numel()
    if grad is None:
        grad = torch.empty(WS_PARAMS, dtype=torch.float32, device=params.device)
    need = int(lib().pcpm_ws_work_floats(b))
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.float32, device=params.device)
    rows = feat.shape[0]
    loss = ctypes.c_double(0.0)
    _check(lib().pcpm_ws_backward(_dev_tensor(params, torch.float32, WS_PARAMS, "params"),
                                  _dev_tensor(feat, torch.float32, rows * WS_FEATURES, "feat"),
                                  _dev_tensor(target, torch.float32, rows, "target"), rows,
                                  _dev_tensor(idx, torch.int64, b, "idx"), b,
                                  _dev_tensor(grad, torch.float32, WS_PARAMS, "grad"),
                                  _dev_tensor(work, torch.float32, name="work"), ctypes.byref(loss),
                                  _stream(stream)))
    return grad, loss.value


def ws_backward_noalloc(params, feat, target, idx, grad, stream=None):
    """pcpm_ws_backward_noalloc: the same gradient with the library's fixed
    scratch (minibatches of at most 16384); returns (grad, loss)."""
    import torch
    b = idx.numel()
    rows = feat.shape[0]
    loss = ctypes.c_double(0.0)
    _check(lib().pcpm_ws_backward_noalloc(_dev_tensor(params, torch.float32, WS_PARAMS, "params"),
                                          _dev_tensor(feat, torch.float32, rows * WS_FEATURES, "feat"),
                                          _dev_tensor(target, torch.float32, rows, "target"), rows,
                                          _dev_tensor(idx, torch.int64, b, "idx"), b,
                                          _dev_tensor(grad, torch.float32, WS_PARAMS, "grad"), ctypes.byref(loss),
                                          _stream(stream)))
    return grad, loss.value


def ws_adam(params, grad, m, v, step: int, lr: float, stream=None):
    import torch
    _check(lib().pcpm_ws_adam(_dev_tensor(params, torch.float32, WS_PARAMS, "params"),
                              _dev_tensor(grad, torch.float32, WS_PARAMS, "grad"),
                              _dev_tensor(m, torch.float32, WS_PARAMS, "m"), _dev_tensor(v, torch.float32, WS_PARAMS, "v"),
                              int(step), float(lr), _stream(stream)))


def ws_targets(pr, stream=None):
    import torch
    n = pr.numel()
    y = torch.empty(n, dtype=torch.float32, device=pr.device)
    _check(lib().pcpm_ws_targets(_dev_tensor(pr, torch.float32, n, "pr"), n, _dev_tensor(y, torch.float32, n, "y"),
                                 _stream(stream)))
    return y
