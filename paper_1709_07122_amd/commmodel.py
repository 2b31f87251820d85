"""Memory-traffic models of Sec. 4 and the byte accounting of the GPU kernels.

Sec. 4.1 (Table 2 notation): n nodes, m edges, k partitions, r = m/|E'|
compression ratio, d_i index bytes, d_v value bytes, c_mr cache-miss ratio of
pull-direction value reads, l cache-line bytes.
"""
from __future__ import annotations


def pdpr_comm(n, m, c_mr, l=64, d_i=4, d_v=4):
    """Eq. 3: bytes per iteration of pull-direction PageRank."""
    return m * (d_i + c_mr * l) + n * (d_i + d_v)


def bvgas_comm(n, m, d_i=4, d_v=4):
    """Eq. 4: bytes per iteration of binning with vertex-centric GAS."""
    return 2 * m * (d_i + d_v) + n * (d_i + 2 * d_v)


def pcpm_comm(n, m, k, r, d_i=4, d_v=4):
    """Eq. 5: bytes per iteration of PCPM over the PNG layout: m(d_i(1+1/r) +
    2 d_v / r) + k^2 d_i + 2 n d_v."""
    return m * (d_i * (1 + 1 / r) + 2 * d_v / r) + k * k * d_i + 2 * n * d_v


def pcpm_comm_bounds(m, d_i=4, d_v=4):
    """Sec. 4.1: with k^2 << n << m, PCPM traffic lies in [m d_i, m(2 d_i + 2 d_v)]
    (r = m/n at best, r = 1 at worst)."""
    return m * d_i, m * (2 * d_i + 2 * d_v)


def bvgas_random_accesses(m, d_v=4, l=64):
    """Sec. 4.2: at most one random DRAM access per cache line of updates."""
    return m * d_v / l


def pcpm_random_accesses(k):
    """Sec. 4.2: at most k bin switches for each of the k partitions."""
    return k * k


def compression_ratio(m, eprime):
    """r = |E| / |E'| (Table 2)."""
    return m / eprime


def gteps(m, seconds_per_iteration):
    """Sec. 5.3: giga edges of the graph per second of one iteration."""
    return m / seconds_per_iteration / 1e9


# ---- byte accounting of this implementation (per launch) ---------------------

TILE = 1024  # destination IDs / PNG edges per stored flag-prefix entry


SRC_BYTES = 2  # PNG source IDs are stored partition-local in 16 bits (flag in bit 15)


def scatter_bytes(n, eprime, nseg, src_bytes=SRC_BYTES, png_order=False):
    """Algorithmic bytes of one scatter pass: ranks and out-degrees of every
    node (8n), the PNG source IDs (src_bytes per PNG edge) and the update
    writes (4E').  With updates in bin order also one write offset per
    non-empty (pair, bin) segment (4 nseg, the k^2 d_i term of Eq. 5) and the
    tile flag prefixes (4E'/1024); in PNG order the writes need neither."""
    extra = 0 if png_order else 4 * nseg + 4 * (eprime // TILE + 1)
    return 8 * n + src_bytes * eprime + extra + 4 * eprime


DID_BYTES = 2  # destination IDs are stored partition-local in 16 bits (flag in bit 15)


def gather_bytes(n, m, eprime, did_bytes=DID_BYTES, nseg=0, png_order=False):
    """Algorithmic bytes of one gather+apply pass: destination IDs
    (did_bytes per edge), tile flag prefixes (4m/1024), updates (4E'), the
    previous ranks for the residual (4n), the new ranks (4n) and the dangling
    bitmask (n/8).  With updates in PNG order also the segment deltas
    (4 nseg) and the segment-flag prefixes (4m/1024)."""
    extra = 4 * nseg + 4 * (m // TILE + 1) if png_order else 0
    return did_bytes * m + 4 * (m // TILE + 1) + 4 * eprime + 8 * n + n // 8 + extra


def iteration_bytes(n, m, eprime, nseg, png_order=False):
    return (scatter_bytes(n, eprime, nseg, png_order=png_order)
            + gather_bytes(n, m, eprime, nseg=nseg, png_order=png_order))


# ---- SpMV over the PNG (Sec. 3.5) -------------------------------------------

def spmv_scatter_bytes(n, eprime, nseg, src_bytes=SRC_BYTES, png_order=False):
    """Scatter of one SpMV: x (4n, no out-degrees), PNG source IDs, the update
    writes, and in bin order the write offsets and tile flag prefixes."""
    return scatter_bytes(n, eprime, nseg, src_bytes, png_order) - 4 * n


def spmv_gather_bytes(n, m, eprime, weighted=True, did_bytes=DID_BYTES, nseg=0, png_order=False):
    """Gather of one SpMV: destination IDs, their weights (4m when weighted,
    stored beside the IDs, Sec. 3.5), tile flag prefixes, updates and y (4n);
    no residual, no dangling mask; in PNG order also the segment deltas and
    segment-flag prefixes."""
    extra = 4 * nseg + 4 * (m // TILE + 1) if png_order else 0
    return did_bytes * m + (4 * m if weighted else 0) + 4 * (m // TILE + 1) + 4 * eprime + 4 * n + extra


def spmv_bytes(n, m, eprime, nseg, weighted=True, png_order=False):
    """Whole SpMV: the scale pass reads x once (4n), then scatter and gather."""
    return (4 * n + spmv_scatter_bytes(n, eprime, nseg, png_order=png_order)
            + spmv_gather_bytes(n, m, eprime, weighted, nseg=nseg, png_order=png_order))
