"""The C-ABI library loads and exports every entry point include/pcpm.h
declares (no device calls: runs without a GPU)."""
import ctypes
import os
import re

import numpy as np

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


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, from a C program built with gcc."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pcpm.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and field
    offsets (a mismatch would pass wrong arguments without any error)."""
    _pcpm = P._pcpm
    for struct, cls in (("pcpm_build_opts_t", _pcpm.BuildOpts), ("pcpm_png_info_t", _pcpm.PngInfo),
                        ("pcpm_kernel_time_t", _pcpm.KernelTime), ("pcpm_tune_entry_t", _pcpm.TuneEntry)):
        fields = [f for f, _ in cls._fields_]
        size, offsets = _c_layout(tmp_path, struct, fields)
        assert ctypes.sizeof(cls) == size, struct
        assert [getattr(cls, f).offset for f in fields] == offsets, struct


def test_null_handles_are_rejected_without_device():
    lib = P.lib()
    assert lib.pcpm_spmv(None, None, None, None) == P.PCPM_ERR_INVALID_ARG
    assert lib.pcpm_png_export_weights(None, None) == P.PCPM_ERR_INVALID_ARG
    assert lib.pcpm_ppr_tile_width(None) == 0


def test_square_csr_pads_rows():
    r = np.array([0, 2, 3], np.int32)  # 2 rows
    c = np.array([1, 4, 0], np.int32)  # 5 columns
    r2, c2 = P.square_csr(r, c, 5)
    assert r2.tolist() == [0, 2, 3, 3, 3, 3] and c2.tolist() == c.tolist()
    r3, _ = P.square_csr(np.array([0, 1, 1, 2], np.int32), np.array([1, 0], np.int32), 2)
    assert r3.tolist() == [0, 1, 1, 2]  # more rows than columns: unchanged


def test_autotune_reads_entries_without_update_order(tmp_path):
    import json
    from paper_1709_07122_amd import autotune
    path = tmp_path / "t.json"
    path.write_text(json.dumps({"k": {"part_log2": 13, "tile_width": 2, "ms_per_iter": 0.5, "build_ms": 3.0,
                                      "table": [], "cached": False}}))
    hit = autotune._load(str(path))["k"]
    res = autotune.TuneResult(**hit)
    assert res.part_log2 == 13 and res.update_order == 0  # 0 lets the build choose
