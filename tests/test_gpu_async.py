"""The batch in caller memory (pc_workspace_bytes + pc_pi_count_batch_async)
on the GPU: the caller owns the queries, the results, the workspace and the
stream, allocated here through the HIP runtime the library itself uses.
Every result equals the synchronous batch (itself pinned to the per-query
path, the oracle and the paper's tables); too small a workspace is refused
before anything is written; a query too large for a round takes the windowed
path during the call and lands in the caller's array like the rest.  Inputs:
x log-uniform from fixed seeds plus edge values, and the batch workload (4096
x log-uniform in [1e8, 1e15])."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SENTINEL = 7
H2D, D2H = 1, 2


def say(*a):
    print(*a, flush=True)


class Hip:
    """The few HIP runtime calls a caller makes, from the runtime that
    libpicount.so is linked against (already loaded with it)."""

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

    def ck(self, rc, what):
        assert rc == 0, f"{what}: HIP error {rc}"

    def malloc(self, nbytes):
        p = C.c_void_p()
        self.ck(self.L.hipMalloc(C.byref(p), max(nbytes, 1)), "hipMalloc")
        self.live.append(p.value)
        return p.value

    def put_u64(self, vals):
        a = np.array(vals, dtype=np.uint64)
        d = self.malloc(a.nbytes)
        self.ck(self.L.hipMemcpy(d, a.ctypes.data, a.nbytes, H2D), "hipMemcpy")
        return d

    def get_u64(self, d, n):
        a = np.zeros(n, dtype=np.uint64)
        self.ck(self.L.hipMemcpy(a.ctypes.data, d, a.nbytes, D2H), "hipMemcpy")
        return [int(v) for v in a]

    def stream(self):
        s = C.c_void_p()
        self.ck(self.L.hipStreamCreate(C.byref(s)), "hipStreamCreate")
        return s.value

    def sync(self, s):
        self.ck(self.L.hipStreamSynchronize(s), "hipStreamSynchronize")

    def free_all(self):
        self.ck(self.L.hipDeviceSynchronize(), "hipDeviceSynchronize")
        for p in self.live:
            self.L.hipFree(p)
        self.live = []


@pytest.fixture
def hip(pc):
    h = Hip()
    yield h
    h.free_all()


def run_async(pc, hip, xs, stream=None, slack=0):
    """pi of xs through the caller-memory path; returns (results, workspace bytes)."""
    n = len(xs)
    need = pc.workspace_bytes(xs)
    d_xs = hip.put_u64(xs)
    d_out = hip.put_u64([SENTINEL] * n)
    ws = hip.malloc(need + slack)
    pc.pi_count_batch_async(d_xs, n, d_out, ws, need + slack, stream)
    hip.sync(stream)
    return hip.get_u64(d_out, n), need


def test_async_equals_sync(pc, hip, paper_pow10):
    rng = np.random.Generator(np.random.PCG64(1503))
    xs = [int(10 ** v) for v in rng.uniform(8, 13, 120)]
    xs += [0, 1, 2, 3, 100, 2**20 - 1, 2**20, 2**20 + 1, 10**9, 10**9, 10**12, 7]
    say("case: async vs sync", len(xs))
    got, need = run_async(pc, hip, xs)
    assert got == pc.pi_count_batch(xs)
    assert got[-12:-7] == [0, 0, 1, 2, 25]
    assert got[-4] == got[-3] == paper_pow10[9]
    assert got[-2] == paper_pow10[12]
    assert need > 0


def test_async_two_calls_one_stream(pc, hip):
    # two batches queued back to back on a stream of the caller's (default
    # priority), the second smaller and with its own workspace; both complete
    a = [int(10 ** v) for v in np.random.Generator(np.random.PCG64(5)).uniform(9, 12, 48)]
    b = a[:9][::-1]
    say("case: async two calls")
    st = hip.stream()
    try:
        outs = []
        for xs in (a, b):
            need = pc.workspace_bytes(xs)
            d_xs, d_out = hip.put_u64(xs), hip.put_u64([SENTINEL] * len(xs))
            ws = hip.malloc(need)
            pc.pi_count_batch_async(d_xs, len(xs), d_out, ws, need, st)
            outs.append(d_out)
        hip.sync(st)
        assert hip.get_u64(outs[0], len(a)) == pc.pi_count_batch(a)
        assert hip.get_u64(outs[1], len(b)) == pc.pi_count_batch(b)
    finally:
        hip.sync(st)
        hip.L.hipStreamDestroy(st)


def test_async_small_workspace_writes_nothing(pc, hip):
    xs = [10**10, 10**11, 5, 10**9]
    say("case: async workspace too small")
    need = pc.workspace_bytes(xs)
    d_xs, d_out = hip.put_u64(xs), hip.put_u64([SENTINEL] * len(xs))
    ws = hip.malloc(need)
    with pytest.raises(pc.PicountError) as e:
        pc.pi_count_batch_async(d_xs, len(xs), d_out, ws, need - 256, None)
    assert e.value.status == pc.PC_ENOMEM
    hip.sync(None)
    assert hip.get_u64(d_out, len(xs)) == [SENTINEL] * len(xs)
    # the same call with the full workspace
    pc.pi_count_batch_async(d_xs, len(xs), d_out, ws, need, None)
    hip.sync(None)
    assert hip.get_u64(d_out, len(xs)) == pc.pi_count_batch(xs)


def test_async_empty_and_small_only(pc, hip):
    say("case: async empty / small only")
    assert pc.workspace_bytes([]) == 0
    pc.pi_count_batch_async(0, 0, 0, 0, 0, None)  # n = 0 touches nothing
    xs = [0, 1, 2, 10, 1000, 2**20 - 1]
    got, need = run_async(pc, hip, xs)
    assert got == [0, 0, 1, 4, 168, pc.pi_count(2**20 - 1)]
    assert need == 256  # the (position, value) pairs only: no round
    with pytest.raises(pc.PicountError) as e:
        pc.pi_count_batch_async(0, 3, 0, 0, 0, None)
    assert e.value.status == pc.PC_EINVAL


def test_async_windowed_query(pc, hip, paper_pow10):
    # pi(10^18): its sieve counts exceed a round's budget, so it is computed
    # windowed during the call and needs no arena in the caller's workspace
    xs = [10**18, 10**10, 10**8]
    say("case: async windowed 1e18")
    assert pc.workspace_bytes(xs[:1]) == 256
    got, _ = run_async(pc, hip, xs)
    assert got == [paper_pow10[18], paper_pow10[10], paper_pow10[8]]


def test_async_batch_workload(pc, hip):
    # the batch workload at full size, against the synchronous batch
    from paper_1503_01839_amd import workloads as W
    xs = W.batch_queries(4096)
    say("case: async batch workload 4096")
    got, need = run_async(pc, hip, xs, slack=4096)
    say("workspace bytes", need)
    assert got == pc.pi_count_batch(xs)
