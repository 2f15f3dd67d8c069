"""CPU-side checks of the HIP library (no GPU needed).

* libpicount.so loads and exports every function include/picount.h declares,
  and the Python binding lists exactly those names.
* The integer helpers the kernels use (division by precomputed reciprocals,
  fp64-estimate quotients, integer roots, the pi-table lookup) compiled for the
  host agree with plain 128-bit arithmetic and a trial-division sieve
  (tests/host/arith_check.hip).
* Calls that need no device answer without one: status strings, wheel size.
"""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "picount.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1503_01839_amd as pc
    if not os.path.exists(pc.LIB_PATH):
        if shutil.which("hipcc") is None:
            pytest.skip("libpicount.so is not built and hipcc is absent")
        from paper_1503_01839_amd import build
        build.build()
    return C.CDLL(pc.LIB_PATH)


def test_header_lists_the_entry_points():
    names = declared_functions()
    for n in ("pc_pi_count", "pc_s2_hard", "pc_p2", "pc_pi_count_batch"):
        assert n in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_1503_01839_amd as pc
    assert sorted(pc.EXPORTS) == declared_functions()


def test_calls_without_device(lib):
    lib.pc_status_str.restype = C.c_char_p
    lib.pc_status_str.argtypes = [C.c_int]
    assert lib.pc_status_str(0) == b"ok"
    assert lib.pc_status_str(1) != lib.pc_status_str(2)
    assert lib.pc_wheel_c() == 6


def test_host_arithmetic(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc is absent")
    exe = tmp_path / "arith_check"
    subprocess.run(["hipcc", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1503_01839_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", "arith_check.hip"), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout


def test_async_argument_checks_without_device(lib):
    # the caller-memory batch: n = 0 and null pointers are answered before
    # any device call
    lib.pc_workspace_bytes.restype = C.c_size_t
    lib.pc_workspace_bytes.argtypes = [C.c_void_p, C.c_size_t]
    lib.pc_pi_count_batch_async.restype = C.c_int
    lib.pc_pi_count_batch_async.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                            C.c_size_t, C.c_void_p]
    lib.pc_last_error.restype = C.c_char_p
    assert lib.pc_workspace_bytes(None, 0) == 0
    assert lib.pc_workspace_bytes(None, 3) == 2**64 - 1
    assert b"null" in lib.pc_last_error()
    assert lib.pc_pi_count_batch_async(None, 0, None, None, 0, None) == 0
    assert lib.pc_pi_count_batch_async(None, 3, None, None, 0, None) == 1  # PC_EINVAL
