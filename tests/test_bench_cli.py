"""bench.py's host-side contract (no GPU): one GPU only, with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_legs():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--no-indegree", "--no-spmv", "--update-order"):
        assert flag in r.stdout


def test_counter_summary_is_matched_to_the_kernel_code():
    """The bench reports counter traffic only while the kernel code is the one
    profiled: comments and layout may change, code may not."""
    sys.path.insert(0, ROOT)
    import bench

    src = "// header\nint f(int x) {  /* twice */ return 2 * x; }\n"
    key = bench.kernel_source_key(src)
    assert bench.kernel_source_key("// other header\nint f(int x) {\n  return 2 * x;  // doubled\n}\n") == key
    assert bench.kernel_source_key("int f(int x) { return 3 * x; }\n") != key
