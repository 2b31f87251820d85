"""PCPM PageRank on AMD MI355X (gfx950).

Python face of libpcpm (see include/pcpm.h): the Partition-Centric Processing
Methodology of Lakhotia, Kannan and Prasanna (arXiv 1709.07122) as
hand-written HIP kernels.  This package only marshals arguments; PyTorch
provides device memory and streams.
"""
from ._pcpm import (EXPORTS, LIB_PATH, PCPM_ERR_DEVICE, PCPM_ERR_GRAPH, PCPM_ERR_INVALID_ARG,
                    PCPM_ERR_NOT_CONVERGED, PCPM_ERR_OOM,
                    PCPM_ERR_NUMERIC, PCPM_ERR_OVERFLOW, PCPM_OK, PNG, PCPMError, PagerankResult, build_png,
                    WS_FEATURES, WS_HIDDEN, WS_PARAMS, iterate, last_error, lib, pagerank, ppr_batch, ppr_tile_width,
                    relabel, spmv, square_csr, graph_hash, tune_cache_clear, hbm_stream, timing_collect, timing_enable, union_csr, ws_adam, ws_backward, ws_backward_noalloc, ws_features,
                    ws_forward, ws_init, ws_predict, ws_targets)
from . import autotune, commmodel, warmstart

__all__ = ["EXPORTS", "LIB_PATH", "PNG", "PCPMError", "PagerankResult", "build_png", "iterate", "pagerank", "ppr_batch", "ppr_tile_width",
           "last_error", "lib", "graph_hash", "tune_cache_clear", "hbm_stream", "relabel", "spmv", "square_csr", "timing_enable", "timing_collect", "union_csr", "autotune", "commmodel", "warmstart",
           "ws_features", "ws_forward", "ws_predict", "ws_init", "ws_backward", "ws_backward_noalloc", "ws_adam", "ws_targets", "WS_FEATURES",
           "WS_HIDDEN", "WS_PARAMS", "PCPM_OK",
           "PCPM_ERR_DEVICE", "PCPM_ERR_GRAPH", "PCPM_ERR_INVALID_ARG", "PCPM_ERR_NOT_CONVERGED", "PCPM_ERR_NUMERIC", "PCPM_ERR_OOM",
           "PCPM_ERR_OVERFLOW"]
