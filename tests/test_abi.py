"""The C-ABI library loads and exports every entry point include/pcpm.h
declares (no device calls: runs without a GPU)."""
import ctypes
import os
import re

import paper_1709_07122_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pcpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pcpm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pcpm_build_png", "pcpm_iterate", "pcpm_pagerank"):
        assert required in names
    assert sorted(P.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1709_07122_amd import _pcpm
    monkeypatch.setattr(_pcpm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_pcpm, "_lib", None)
    try:
        _pcpm.lib()
    except ImportError as e:
        assert "missing" in str(e)
    else:
        raise AssertionError("loading a missing library must raise")


def test_host_only_calls_without_device():
    lib = P.lib()
    lib.pcpm_timing_enable(0)
    assert lib.pcpm_timing_collect(None, 0) == 0
    # NULL-handle calls return INVALID_ARG without touching a device
    info = P._pcpm.PngInfo()
    assert lib.pcpm_png_info(None, ctypes.byref(info)) == P.PCPM_ERR_INVALID_ARG
    assert "NULL" in P.last_error()
    lib.pcpm_png_free(None)
