"""The traffic and random-access models of Sec. 4 against the paper's numbers."""
import pytest

from paper_1709_07122_amd import commmodel as cm


def test_random_access_example_of_sec4_2():
    """kron: d_v = 4 B, l = 64 B, k = 512, m = 1070M (Fig. 6 parameters):
    BVGAS about 66.9M random accesses, PCPM about 0.26M."""
    assert round(cm.bvgas_random_accesses(1070e6, 4, 64) / 1e6, 1) == 66.9
    assert round(cm.pcpm_random_accesses(512) / 1e6, 2) == 0.26


@pytest.mark.parametrize("m,eprime,r", [(463, 243.8, 1.9), (623.1, 347.7, 1.79), (992.8, 118.1, 8.4),
                                        (1047.9, 342.7, 3.06), (1468.4, 722.4, 2.03), (1937.5, 976.9, 1.98),
                                        (463, 157.4, 2.94), (623.1, 166.7, 3.73), (1937.5, 366.2, 5.29)])
def test_table6_compression_ratios(m, eprime, r):
    """Table 6 (kron row with the edge count of Table 4, 1047.9M)."""
    assert round(cm.compression_ratio(m, eprime), 2) == pytest.approx(r, abs=0.011)


def test_eq5_limits_and_bounds():
    n, m, k = 33.5e6, 1070e6, 512
    lo, hi = cm.pcpm_comm_bounds(m)
    # r = 1: every edge its own message; r = m/n: one message per node
    worst = cm.pcpm_comm(n, m, k, 1.0)
    best = cm.pcpm_comm(n, m, k, m / n)
    assert worst == pytest.approx(m * 16 + k * k * 4 + 8 * n)
    assert lo <= best < worst <= hi + k * k * 4 + 8 * n
    assert cm.pcpm_comm(n, m, k, 3.06) < cm.bvgas_comm(n, m)
    # Eq. 3 with every value read missing the cache, and with cold misses only
    assert cm.pdpr_comm(n, m, 1.0) == pytest.approx(m * (4 + 64) + n * 8)
    assert cm.pdpr_comm(n, m, n * 4 / (m * 64)) == pytest.approx(m * 4 + n * 4 + n * 8)


def test_gteps_definition():
    """Sec. 5.3: GTEPS = edges of the graph / time of one iteration; kron at
    0.25 s per iteration (Table 5) gives about 4.19."""
    assert round(cm.gteps(1047.93e6, 0.25), 2) == 4.19


def test_implementation_bytes_cover_eq5():
    n, m, ep, k = 1 << 24, 263_400_000, 174_000_000, 1024
    ours = cm.iteration_bytes(n, m, ep, k * k)
    # Eq. 5 with the destination IDs (its m d_i term) and the PNG source IDs
    # (its m d_i / r term) at the 2 bytes they are stored in
    eq5 = cm.pcpm_comm(n, m, k, m / ep) - (4 - cm.DID_BYTES) * m - (4 - cm.SRC_BYTES) * ep
    # the same terms plus 8 B per node (residual read, out-degrees) and the
    # tile prefixes; never less than that
    assert eq5 < ours < eq5 + 8.5 * n + 4 * (m + ep) / 1024 + 8
    assert cm.gather_bytes(n, m, ep, did_bytes=4) - cm.gather_bytes(n, m, ep) == 2 * m


def test_spmv_bytes_add_up():
    n, m, ep, nseg = 1000, 16000, 9000, 300
    s = cm.spmv_scatter_bytes(n, ep, nseg)
    g = cm.spmv_gather_bytes(n, m, ep)
    assert s == 4 * n + 2 * ep + 4 * nseg + 4 * (ep // 1024 + 1) + 4 * ep
    assert g == 2 * m + 4 * m + 4 * (m // 1024 + 1) + 4 * ep + 4 * n
    assert cm.spmv_gather_bytes(n, m, ep, weighted=False) == g - 4 * m
    assert cm.spmv_bytes(n, m, ep, nseg) == 4 * n + s + g


def test_png_order_moves_the_offsets_to_the_gather():
    n, m, ep, nseg = 1000, 16000, 9000, 300
    assert cm.scatter_bytes(n, ep, nseg) - cm.scatter_bytes(n, ep, nseg, png_order=True) == 4 * nseg + 4 * (ep // 1024 + 1)
    assert cm.gather_bytes(n, m, ep, nseg=nseg, png_order=True) - cm.gather_bytes(n, m, ep) == 4 * nseg + 4 * (m // 1024 + 1)
    assert cm.iteration_bytes(n, m, ep, nseg, png_order=True) == (cm.scatter_bytes(n, ep, nseg, png_order=True)
                                                                  + cm.gather_bytes(n, m, ep, nseg=nseg, png_order=True))
