"""The quotient helpers of the kernels (pc_device.h) run on the GPU over 10^8
seeded random pairs shaped to each helper's domain plus edge pairs: pc_quot32,
pc_quot31, pc_quot31r, pc_quot_in, pc_div_small_q, pc_div, the fp64
reciprocal pc_rcp_f64, and the helpers of x above 2^64: pc_div_wide32,
pc_div_u128_32, pc_div_wide, pc_div_small_qd, pc_quot_in64 and
pc_isqrt_wide.  Every quotient is checked exactly against
q d <= n < (q + 1) d in 128-bit integer arithmetic
(tests/device/div_check.hip)."""
import ctypes as C
import os

import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "device", "libdivcheck.so")
NAMES = ("pc_quot32", "pc_quot_in", "pc_div_small_q", "pc_div", "pc_rcp_f64", "pc_quot31r",
         "pc_quot31", "pc_div_wide32", "pc_div_wide", "pc_quot_in64", "pc_div_u128_32",
         "pc_div_small_qd", "pc_isqrt_wide")


@pytest.mark.parametrize("seed", [1503, 1839])
def test_quotient_helpers_exact(pc, seed):
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is missing: run __graft_entry__.build()")
    pc.lib()  # the HIP runtime the library uses is loaded first
    L = C.CDLL(LIB)
    L.pc_div_check.argtypes = [C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p]
    L.pc_div_check.restype = C.c_int
    fails = (C.c_uint64 * len(NAMES))()
    first = (C.c_uint64 * len(NAMES))()
    print("case: device quotients, 10^8 pairs, seed", seed, flush=True)
    assert L.pc_div_check(10**8, seed, fails, first) == 0
    bad = {NAMES[k]: (fails[k], first[k]) for k in range(len(NAMES)) if fails[k]}
    assert not bad, f"failures (count, first pair index): {bad}"
