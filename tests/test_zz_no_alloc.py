"""The allocation-free batch (pc_pi_count_batch_noalloc) on the GPU, through
the C ABI: its results equal those of the caller-memory batch
(pc_pi_count_batch_async, the existing entry point it is a variant of) on the
same device arrays, for two calls in a row, the second with fewer and smaller
queries; requests it cannot serve without allocating are refused without
writing anything.  Inputs: x log-uniform from fixed seeds plus edge values."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SENTINEL = 7
H2D, D2H = 1, 2


def say(*a):
    print(*a, flush=True)


class Hip:
    """hipMalloc / hipMemcpy from the runtime libpicount.so is linked against,
    for the caller's own arrays (the entry point itself allocates nothing)."""

    def __init__(self):
        L = C.CDLL("libamdhip64.so.7")
        L.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        L.hipFree.argtypes = [C.c_void_p]
        L.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        L.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
        L.hipStreamSynchronize.argtypes = [C.c_void_p]
        L.hipStreamDestroy.argtypes = [C.c_void_p]
        self.L = L
        self.live = []

    def malloc(self, nbytes):
        p = C.c_void_p()
        assert self.L.hipMalloc(C.byref(p), max(nbytes, 1)) == 0
        self.live.append(p.value)
        return p.value

    def put(self, vals):
        a = np.array(vals, dtype=np.uint64)
        d = self.malloc(a.nbytes)
        assert self.L.hipMemcpy(d, a.ctypes.data, a.nbytes, H2D) == 0
        return d

    def get(self, d, n):
        a = np.zeros(n, dtype=np.uint64)
        assert self.L.hipMemcpy(a.ctypes.data, d, a.nbytes, D2H) == 0
        return [int(v) for v in a]

    def free_all(self):
        assert self.L.hipDeviceSynchronize() == 0
        for p in self.live:
            self.L.hipFree(p)
        self.live = []


@pytest.fixture
def hip(pc):
    h = Hip()
    yield h
    h.free_all()


def noalloc(pc):
    L = pc.lib()
    f = L.pc_pi_count_batch_noalloc
    f.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
    f.restype = C.c_int
    return f


def via_async(pc, hip, xs, stream):
    need = pc.workspace_bytes(xs)  # also builds the tables these x need
    d_xs, d_out = hip.put(xs), hip.put([SENTINEL] * len(xs))
    ws = hip.malloc(need)
    pc.pi_count_batch_async(d_xs, len(xs), d_out, ws, need, stream)
    assert hip.L.hipStreamSynchronize(stream) == 0
    return hip.get(d_out, len(xs))


def via_noalloc(pc, hip, xs, stream):
    d_xs, d_out = hip.put(xs), hip.put([SENTINEL] * len(xs))
    st = noalloc(pc)(d_xs, len(xs), d_out, stream)
    assert st == pc.PC_OK, pc.lib().pc_last_error().decode()
    return hip.get(d_out, len(xs))


def test_noalloc_equals_async_two_calls(pc, hip, paper_pow10):
    rng = np.random.Generator(np.random.PCG64(1503))
    a = [int(10 ** v) for v in rng.uniform(8, 15, 300)]
    a += [0, 1, 2, 100, 2**20 - 1, 2**20, 10**9, 10**9, 10**12, 10**15]
    b = [int(10 ** v) for v in np.random.Generator(np.random.PCG64(5)).uniform(8, 11, 37)]
    st = C.c_void_p()
    assert hip.L.hipStreamCreate(C.byref(st)) == 0
    try:
        want_a = via_async(pc, hip, a, st.value)
        want_b = via_async(pc, hip, b, st.value)
        say("case: noalloc first call", len(a))
        got_a = via_noalloc(pc, hip, a, st.value)
        assert got_a == want_a
        assert got_a[-4] == got_a[-3] == paper_pow10[9]
        assert got_a[-2:] == [paper_pow10[12], paper_pow10[15]]
        say("case: noalloc second, smaller call", len(b))
        got_b = via_noalloc(pc, hip, b, st.value)
        assert got_b == want_b
        say("case: noalloc null stream")
        assert via_noalloc(pc, hip, b[:5], None) == want_b[:5]
    finally:
        hip.L.hipStreamSynchronize(st.value)
        hip.L.hipStreamDestroy(st.value)


def test_noalloc_refusals_write_nothing(pc, hip):
    f = noalloc(pc)
    assert f(None, 0, None, None) == pc.PC_OK          # n = 0 touches nothing
    assert f(None, 3, None, None) == pc.PC_EINVAL
    # too large for a round of the scratch array
    xs = [10**9, 10**18]
    pc.workspace_bytes(xs)
    d_xs, d_out = hip.put(xs), hip.put([SENTINEL] * 2)
    say("case: noalloc refuses 1e18")
    assert f(d_xs, 2, d_out, None) == pc.PC_ERANGE
    assert hip.get(d_out, 2) == [SENTINEL] * 2
    # tables not covering the query: none of the library's tables reaches y
    # of 1e19 until a call builds them
    pc.shutdown()
    d_xs = hip.put([10**12])
    d_out = hip.put([SENTINEL])
    say("case: noalloc refuses without tables")
    assert f(d_xs, 1, d_out, None) == pc.PC_ERANGE
    assert hip.get(d_out, 1) == [SENTINEL]
