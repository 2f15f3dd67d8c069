"""MI355X (gfx950) prime counting by the combinatorial method.

Thin ctypes binding over ``libpicount.so`` (C ABI in ``include/picount.h``):
argument marshalling only.  Every step of the computation runs in the
library's HIP kernels; this module raises if the library is missing rather
than computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpicount.so")

PC_OK, PC_EINVAL, PC_ERANGE, PC_ENOMEM, PC_EDEVICE, PC_EINTERNAL = range(6)
FLAG_TWO_PASS = 1
FLAG_NO_BATCH_LARGE = 2
FLAG_REBUILD_TABLES = 4
FLAG_NO_SMALL_SEGMENTS = 8
FLAG_NO_GRAPH = 16
FLAG_BATCH_SEQUENTIAL = 32
FLAG_SEEDED = 64
TABLE_PRIMES, TABLE_PI, TABLE_MULPF = 1, 2, 3

EXPORTS = ["pc_pi_count", "pc_pi_count_ex", "pc_pi_count_wide", "pc_s2_hard", "pc_decompose",
           "pc_p2",
           "pc_pi_count_batch", "pc_pi_count_batch_ex", "pc_workspace_bytes",
           "pc_pi_count_batch_async", "pc_pi_count_batch_noalloc", "pc_serve", "pc_read_table",
           "pc_phi_seed", "pc_wheel_c",
           "pc_status_str", "pc_last_error", "pc_shutdown"]


class PicountError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"picount status {status}: {msg}")
        self.status = status


class I128(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_int64)]

    def value(self) -> int:
        return (self.hi << 64) + self.lo


class Config(C.Structure):
    _fields_ = [("alpha", C.c_double), ("segment_kib", C.c_uint32), ("wg_size", C.c_uint32),
                ("tile_leaves", C.c_uint32), ("flags", C.c_uint32),
                ("carry_budget", C.c_uint64), ("small_span", C.c_uint32),
                ("small_kib", C.c_uint32)]


class _Result(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("x", "y", "a", "c", "z", "bmax", "pi")] + \
               [(n, I128) for n in ("s1", "s2_trivial", "s2_easy", "s2_hard", "p2", "phi")] + \
               [(n, C.c_uint64) for n in ("n_s1", "n_trivial", "n_easy", "n_hard", "n_p2",
                                          "segments", "tiles", "windows", "segment_bits",
                                          "small_segments", "crossings", "device_bytes")] + \
               [(n, C.c_uint32) for n in ("sieve_launches", "scan_launches")] + \
               [(n, C.c_double) for n in ("ms_total", "ms_tables", "ms_leaves", "ms_sieve",
                                          "ms_k_sieve", "ms_k_scan", "ms_k_easy", "ms_k_s1")] + \
               [("n_easy_items", C.c_uint64), ("x_hi", C.c_uint64), ("pi_hi", C.c_uint64),
                ("ms_k_seed", C.c_double)]


@dataclass
class Result:
    x: int
    y: int
    a: int
    c: int
    z: int
    bmax: int
    pi: int
    s1: int
    s2_trivial: int
    s2_easy: int
    s2_hard: int
    p2: int
    phi: int
    n_s1: int
    n_trivial: int
    n_easy: int
    n_hard: int
    n_p2: int
    segments: int
    tiles: int
    windows: int
    segment_bits: int
    small_segments: int
    crossings: int
    device_bytes: int
    sieve_launches: int
    scan_launches: int
    ms_total: float
    ms_tables: float
    ms_leaves: float
    ms_sieve: float
    ms_k_sieve: float
    ms_k_scan: float
    ms_k_easy: float
    ms_k_s1: float
    n_easy_items: int
    x_hi: int
    pi_hi: int
    ms_k_seed: float

class ServeConfig(C.Structure):
    _fields_ = [("max_inflight", C.c_uint32), ("max_round", C.c_uint32),
                ("mem_budget", C.c_uint64), ("alpha", C.c_double), ("flags", C.c_uint32),
                ("pad", C.c_uint32)]


class ServeStats(C.Structure):
    _fields_ = [("wall_s", C.c_double)] + [(n, C.c_uint64) for n in (
        "rounds", "windowed", "max_round_size", "max_inflight_seen", "device_bytes")]


_lib = None


def lib():
    """Load libpicount.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(or python -m paper_1503_01839_amd.build)")
        L = C.CDLL(LIB_PATH)
        u64, P = C.c_uint64, C.POINTER
        L.pc_pi_count.argtypes = [u64, C.c_double, P(u64)]
        L.pc_pi_count_ex.argtypes = [u64, P(Config), P(_Result)]
        L.pc_pi_count_wide.argtypes = [u64, u64, P(Config), P(_Result)]
        L.pc_s2_hard.argtypes = [u64, u64, u64, P(I128)]
        L.pc_decompose.argtypes = [u64, u64, P(Config), P(_Result)]
        L.pc_p2.argtypes = [u64, u64, P(u64)]
        L.pc_pi_count_batch.argtypes = [P(u64), C.c_size_t, P(u64)]
        L.pc_pi_count_batch_ex.argtypes = [P(u64), C.c_size_t, P(Config), P(u64)]
        L.pc_serve.argtypes = [P(u64), P(C.c_double), C.c_size_t, P(ServeConfig), P(u64),
                               P(C.c_double), P(ServeStats)]
        L.pc_workspace_bytes.argtypes = [P(u64), C.c_size_t]
        L.pc_workspace_bytes.restype = C.c_size_t
        L.pc_pi_count_batch_async.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                              C.c_size_t, C.c_void_p]
        L.pc_pi_count_batch_noalloc.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
        for f in ("pc_pi_count", "pc_pi_count_ex", "pc_pi_count_wide", "pc_s2_hard",
                  "pc_decompose", "pc_p2",
                  "pc_pi_count_batch", "pc_pi_count_batch_ex", "pc_pi_count_batch_async",
                  "pc_pi_count_batch_noalloc", "pc_serve"):
            getattr(L, f).restype = C.c_int
        L.pc_read_table.argtypes = [C.c_int, u64, u64, C.c_void_p]
        L.pc_read_table.restype = C.c_int
        L.pc_phi_seed.argtypes = [u64, C.c_uint32, C.c_uint32, C.c_void_p]
        L.pc_phi_seed.restype = C.c_int
        L.pc_wheel_c.restype = C.c_int
        L.pc_status_str.argtypes = [C.c_int]
        L.pc_status_str.restype = C.c_char_p
        L.pc_last_error.restype = C.c_char_p
        L.pc_shutdown.restype = None
        _lib = L
    return _lib


def _check(st: int):
    if st != PC_OK:
        L = lib()
        raise PicountError(st, f"{L.pc_status_str(st).decode()}: {L.pc_last_error().decode()}")


def _config(alpha=0.0, segment_kib=0, wg_size=0, tile_leaves=0, flags=0, carry_budget=0,
            small_span=0, small_kib=0):
    return Config(float(alpha), segment_kib, wg_size, tile_leaves, flags, carry_budget,
                  small_span, small_kib)


def _result(r: _Result) -> Result:
    vals = {}
    for name, _ in _Result._fields_:
        v = getattr(r, name)
        vals[name] = v.value() if isinstance(v, I128) else v
    return Result(**vals)


def pi_count(x: int, alpha: float = 0.0) -> int:
    """pi(x), 0 <= x < 2^64."""
    out = C.c_uint64(0)
    _check(lib().pc_pi_count(x, float(alpha), C.byref(out)))
    return out.value


def pi_count_ex(x: int, **cfg) -> Result:
    r = _Result()
    c = _config(**cfg)
    _check(lib().pc_pi_count_ex(x, C.byref(c), C.byref(r)))
    return _result(r)


def pi_count_wide(x: int, **cfg) -> Result:
    """pi(x) and its decomposition for 0 <= x <= 2^72 (x may exceed 2^64): the
    result's x and pi fields are full integers (x_hi and pi_hi keep the high
    words the C ABI returns)."""
    if not 0 <= x <= 1 << 72:
        raise ValueError("x must satisfy 0 <= x <= 2^72")
    r = _Result()
    c = _config(**cfg)
    _check(lib().pc_pi_count_wide(x & ((1 << 64) - 1), x >> 64, C.byref(c), C.byref(r)))
    res = _result(r)
    res.x = (res.x_hi << 64) | res.x
    res.pi = (res.pi_hi << 64) | res.pi
    return res


def decompose(x: int, y: int, **cfg) -> Result:
    """S1, S2 (trivial/easy/hard), P2, phi(x, a) and pi(x) for one explicit y."""
    r = _Result()
    c = _config(**cfg)
    _check(lib().pc_decompose(x, y, C.byref(c), C.byref(r)))
    return _result(r)


def s2_hard(x: int, y: int, a: int) -> int:
    out = I128()
    _check(lib().pc_s2_hard(x, y, a, C.byref(out)))
    return out.value()


def p2(x: int, y: int) -> int:
    out = C.c_uint64(0)
    _check(lib().pc_p2(x, y, C.byref(out)))
    return out.value


def pi_count_batch(xs, **cfg) -> list[int]:
    xs = list(xs)
    n = len(xs)
    arr = (C.c_uint64 * max(n, 1))(*xs)
    out = (C.c_uint64 * max(n, 1))()
    if cfg:
        c = _config(**cfg)
        _check(lib().pc_pi_count_batch_ex(arr, n, C.byref(c), out))
    else:
        _check(lib().pc_pi_count_batch(arr, n, out))
    return list(out[:n])


SIZE_MAX = 2**64 - 1


def workspace_bytes(xs) -> int:
    """Device bytes of workspace pi_count_batch_async needs for these x values."""
    xs = list(xs)
    n = len(xs)
    arr = (C.c_uint64 * max(n, 1))(*xs)
    v = lib().pc_workspace_bytes(arr, n)
    if v == SIZE_MAX:
        raise PicountError(-1, lib().pc_last_error().decode())
    return v


def _addr(v) -> int:
    """A device address: a tensor's data_ptr(), a stream's handle, or an int."""
    if v is None:
        return 0
    for attr in ("data_ptr", "cuda_stream"):
        a = getattr(v, attr, None)
        if a is not None:
            return a() if callable(a) else a
    return int(v)


def pi_count_batch_async(d_xs, n: int, d_out, d_ws, ws_bytes: int, stream=None) -> None:
    """out[i] = pi(xs[i]) in caller device memory, queued on `stream`.  Each
    pointer argument is a device address, or a tensor (its data_ptr()); the
    stream is a handle or a torch stream (its cuda_stream); None is the null
    stream."""
    _check(lib().pc_pi_count_batch_async(_addr(d_xs), n, _addr(d_out), _addr(d_ws), ws_bytes,
                                         _addr(stream)))


def pi_count_batch_noalloc(d_xs, n: int, d_out, stream=None) -> None:
    """out[i] = pi(xs[i]) in caller device memory with no allocation (the
    library's fixed scratch array as workspace; the tables must already cover
    these x); returns once out is complete.  Pointer arguments as in
    pi_count_batch_async."""
    _check(lib().pc_pi_count_batch_noalloc(_addr(d_xs), n, _addr(d_out), _addr(stream)))


def serve(xs, arrivals, max_inflight=0, max_round=0, mem_budget=0, alpha=0.0, flags=0):
    """Replay an open-loop request stream (x values, arrival times in seconds)
    in real time with continuous batching; returns (pi values, latencies in
    seconds, stats dict)."""
    xs = list(xs)
    arrivals = [float(t) for t in arrivals]
    n = len(xs)
    if len(arrivals) != n:
        raise ValueError("xs and arrivals differ in length")
    if n == 0:
        return [], [], {}
    xa = (C.c_uint64 * n)(*xs)
    ta = (C.c_double * n)(*arrivals)
    out = (C.c_uint64 * n)()
    lat = (C.c_double * n)()
    st = ServeStats()
    cfg = ServeConfig(max_inflight, max_round, mem_budget, float(alpha), flags, 0)
    _check(lib().pc_serve(xa, ta, n, C.byref(cfg), out, lat, C.byref(st)))
    stats = {f: getattr(st, f) for f, _ in ServeStats._fields_}
    return list(out), list(lat), stats


def read_table(which: int, lo: int, n: int):
    """Entries lo .. lo + n - 1 of a shared device table (TABLE_PRIMES: p_k,
    TABLE_PI: pi(v), TABLE_MULPF: mu(v) * lpf(v)) as a numpy array."""
    import numpy as np
    dt = {TABLE_PRIMES: np.uint32, TABLE_PI: np.uint64, TABLE_MULPF: np.int32}.get(which)
    if dt is None:
        raise ValueError(f"unknown table {which}")
    out = np.zeros(max(n, 1), dtype=dt)
    _check(lib().pc_read_table(which, lo, n, out.ctypes.data))
    return out[:n]


def phi_seed(m: int, b_hi: int, c: int = 6):
    """phi(m, b) for c <= b <= b_hi (numpy uint64, entry b - c), computed on the
    device as the seeds of a sieve started at m (Section 4)."""
    import numpy as np
    out = np.zeros(b_hi - c + 1 if b_hi >= c else 1, dtype=np.uint64)
    _check(lib().pc_phi_seed(m, c, b_hi, out.ctypes.data))
    return out


def wheel_c() -> int:
    return lib().pc_wheel_c()


def shutdown() -> None:
    lib().pc_shutdown()
