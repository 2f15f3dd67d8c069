"""Micro-benchmarks of the GPU's peaks behind the sieve's rooflines
(tests/device/peaks.hip): LDS atomic AND with return in three address
patterns (consecutive words, the crossing pattern, random words), 64-bit
multiply-high, and a device copy.  The figures go to the test's output; the
test checks only that each is positive and of a plausible order (a broken
kernel, not a slow one, fails it)."""
import ctypes as C
import os

import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "device", "libpeaks.so")


def test_peaks():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is missing: run __graft_entry__.build()")
    import paper_1503_01839_amd as pc
    pc.lib()  # the HIP runtime the library uses is loaded first
    L = C.CDLL(LIB)
    L.pc_peaks.restype = C.c_int
    L.pc_peaks.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(C.c_double),
                           C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lds = (C.c_double * 3)()
    mulhi, copy = C.c_double(), C.c_double()
    blocks, iters = 256 * 4, 4096
    print(f"case: peaks, {blocks} workgroups of 512 threads, {iters} steps", flush=True)
    assert L.pc_peaks(blocks, iters, 1 << 30, lds, C.byref(mulhi), C.byref(copy)) == 0
    names = ("consecutive words", "crossing pattern", "random words")
    for n, v in zip(names, lds):
        print(f"LDS atomic AND with return, {n}: {v / 1e9:.1f} G/s", flush=True)
    print(f"64-bit multiply-high: {mulhi.value / 1e12:.2f} T/s", flush=True)
    print(f"device copy: {copy.value / 1e12:.2f} TB/s (read + written)", flush=True)
    assert all(v > 1e10 for v in lds)
    assert mulhi.value > 1e11 and copy.value > 1e11
