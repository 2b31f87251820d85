"""Failure handling forced from the host: sizes past the 31-bit limits return
PCPM_ERR_OVERFLOW before any device work, and device memory exhausted by the
caller gives PCPM_ERR_OOM, after which the library works again."""
import ctypes

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


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_sizes_past_31_bits_overflow():
    lib = P.lib()
    out = ctypes.c_void_p()
    for n, m in ((1 << 31, 0), (5, 1 << 31)):
        rc = lib.pcpm_build_png(n, m, None, None, None, _stream(), ctypes.byref(out))
        assert rc == P.PCPM_ERR_OVERFLOW and not out.value
        rc = lib.pcpm_relabel(n, m, None, None, 0, None, None, None, _stream())
        assert rc == P.PCPM_ERR_OVERFLOW


def test_out_of_device_memory_then_recovery():
    r, c = graphgen.rmat(20, 16, seed=9, relabel="random")
    rt = torch.from_numpy(np.ascontiguousarray(r)).cuda()
    ct = torch.from_numpy(np.ascontiguousarray(c)).cuda()
    n, m = len(r) - 1, len(c)
    outs = torch.empty(2 * n + 1 + m, dtype=torch.int32, device="cuda")  # relabel outputs, allocated beforehand
    torch.cuda.synchronize()
    hog = []  # the caller takes all but ~64 MB of device memory, in pieces of at most 8 GB
    while True:
        free, _ = torch.cuda.mem_get_info()
        if free <= (64 << 20) + (4 << 20):
            break
        hog.append(torch.empty(min(free - (64 << 20), 8 << 30), dtype=torch.uint8, device="cuda"))
    try:
        with pytest.raises(P.PCPMError) as ei:
            P.build_png(rt, ct)
        assert ei.value.status == P.PCPM_ERR_OOM
        vp = lambda t, o=0: ctypes.c_void_p(t.data_ptr() + 4 * o)
        rc = P.lib().pcpm_relabel(n, m, vp(rt), vp(ct), 0, vp(outs), vp(outs, n), vp(outs, 2 * n + 1), _stream())
        assert rc == P.PCPM_ERR_OOM
    finally:
        del hog
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    png = P.build_png(rt, ct)
    res = P.pagerank(png, d=0.85, tol=0.0, max_iters=10)
    o = oracle.pagerank(r, c, d=0.85, iters=10)
    assert np.abs(res.pr.cpu().numpy().astype(np.float64) - o.x).sum() <= 1e-5
