"""Plain CPU reference ("oracle") for the combinatorial pi(x) method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never imports,
links or calls it, and the two share no source.

The arithmetic lives in ``oracle.c`` (plain C, exact integers, signed 128-bit
sums); this module compiles it with gcc into ``liboracle.so`` and wraps it
with ctypes.  Formulas and the sections of the paper they follow are listed
at the top of ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class I128(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_int64)]

    def value(self) -> int:
        return (self.hi << 64) + self.lo


class _Decomp(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("x", "y", "a", "c", "z", "bmax")] + \
               [(n, I128) for n in ("s1", "s2t", "s2e", "s2h", "p2", "phi")] + \
               [(n, C.c_uint64) for n in ("n_s1", "n_trivial", "n_easy", "n_hard", "n_p2",
                                          "phi_nodes")]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        u64 = C.c_uint64
        L.or_isqrt.argtypes = [u64]
        L.or_isqrt.restype = u64
        L.or_icbrt.argtypes = [u64]
        L.or_icbrt.restype = u64
        L.or_pi_brute.argtypes = [u64]
        L.or_pi_brute.restype = u64
        L.or_primes.argtypes = [u64, C.POINTER(C.c_uint32), u64]
        L.or_primes.restype = u64
        L.or_phi.argtypes = [u64, u64, u64, C.POINTER(u64)]
        L.or_phi.restype = I128
        L.or_phi_direct.argtypes = [u64, u64]
        L.or_phi_direct.restype = u64
        L.or_phi_column.argtypes = [u64, u64, C.c_void_p]
        L.or_phi_column.restype = C.c_int
        L.or_p2.argtypes = [u64, u64]
        L.or_p2.restype = I128
        L.or_p2_brute.argtypes = [u64, u64]
        L.or_p2_brute.restype = u64
        P = C.POINTER(I128)
        L.or_decompose.argtypes = [u64, u64, u64, C.c_int, C.c_int, C.c_int, u64,
                                   C.POINTER(_Decomp), P, P, P, P, u64]
        L.or_decompose.restype = C.c_int
        L.or_leaf_sample.argtypes = [u64, u64, u64, u64, u64, u64, u64, C.POINTER(_Decomp)]
        L.or_leaf_sample.restype = C.c_int
        L.or_s1_p2.argtypes = [u64, u64, u64, C.POINTER(_Decomp)]
        L.or_s1_p2.restype = C.c_int
        L.or_mu_lpf.argtypes = [u64, C.c_void_p, C.c_void_p]
        L.or_mu_lpf.restype = C.c_int
        L.or_pi_meissel.argtypes = [u64, u64, u64]
        L.or_pi_meissel.restype = u64
        _lib = L
    return _lib


def isqrt(n: int) -> int:
    return lib().or_isqrt(n)


def icbrt(n: int) -> int:
    return lib().or_icbrt(n)


def pi_brute(n: int) -> int:
    """pi(n) by the sieve of Eratosthenes (§1)."""
    return lib().or_pi_brute(n)


def primes(n: int) -> list[int]:
    cnt = lib().or_primes(n, None, 0)
    buf = (C.c_uint32 * max(cnt, 1))()
    lib().or_primes(n, buf, cnt)
    return list(buf[:cnt])


def mu_lpf(N: int):
    """(mu, lpf) for 0 <= n <= N as numpy arrays (int8, uint32), by a plain
    factor sieve; lpf is 0 for n < 2."""
    import numpy as np
    mu = np.zeros(N + 1, dtype=np.int8)
    lpf = np.zeros(N + 1, dtype=np.uint32)
    if lib().or_mu_lpf(N, mu.ctypes.data, lpf.ctypes.data) != 0:
        raise ValueError(f"or_mu_lpf({N}) failed")
    return mu, lpf


def phi(u: int, b: int, c: int = 6) -> int:
    """phi(u, b) by the recurrence eq. (4.1) (wheel base case for b <= c)."""
    nodes = C.c_uint64(0)
    return lib().or_phi(u, b, c, C.byref(nodes)).value()


def phi_direct(u: int, b: int) -> int:
    """phi(u, b) by testing every n <= u against the first b primes."""
    return lib().or_phi_direct(u, b)


def phi_column(m: int, b_hi: int):
    """phi(m, b) for 0 <= b <= b_hi (numpy uint64), counted from the definition."""
    import numpy as np
    out = np.zeros(b_hi + 1, dtype=np.uint64)
    if lib().or_phi_column(m, b_hi, out.ctypes.data) != 0:
        raise MemoryError(f"or_phi_column({m})")
    return out


def p2(x: int, y: int) -> int:
    """P2(x, pi(y)) from one sieve of [0, x/(y+1)]."""
    return lib().or_p2(x, y).value()


def p2_brute(x: int, y: int) -> int:
    """P2 by factoring every n <= x (tiny x only)."""
    return lib().or_p2_brute(x, y)


@dataclass
class Decomp:
    x: int
    y: int
    a: int
    c: int
    z: int
    bmax: int
    s1: int
    s2t: int
    s2e: int
    s2h: int
    p2: int
    phi: int
    n_s1: int
    n_trivial: int
    n_easy: int
    n_hard: int
    n_p2: int
    phi_nodes: int
    per_b_hard: list | None = None
    per_b_trivial: list | None = None
    per_b_easy: list | None = None
    per_seg_hard: list | None = None

    @property
    def pi(self) -> int:
        """Meissel's identity with phi = S1 + S2."""
        return self.s1 + self.s2t + self.s2e + self.s2h + self.a - 1 - self.p2


HARD_NONE, HARD_SIEVE, HARD_IDENTITY, HARD_BOTH = 0, 1, 2, 3


def decompose(x: int, y: int, c: int = 6, hard: int = HARD_SIEVE, want_phi: bool = False,
              want_p2: bool = True, seglen: int = 0, per_b: bool = False,
              nseg: int = 0) -> Decomp:
    """S1, S2 (trivial/easy/hard), P2 and optionally phi(x, a) for one (x, y, c)."""
    L = lib()
    D = _Decomp()
    a = pi_brute(y) if per_b else 0
    arrs = [None, None, None]
    if per_b:
        arrs = [(I128 * (a + 1))() for _ in range(3)]
    seg = (I128 * nseg)() if nseg else None
    rc = L.or_decompose(x, y, c, hard, int(want_phi), int(want_p2), seglen, C.byref(D),
                        arrs[0], arrs[1], arrs[2], seg, nseg)
    if rc != 0:
        raise ValueError(f"or_decompose({x}, {y}, {c}) failed with code {rc}")
    vals = {f: getattr(D, f) for f, _ in _Decomp._fields_}
    for k in ("s1", "s2t", "s2e", "s2h", "p2", "phi"):
        vals[k] = vals[k].value()
    out = Decomp(**vals)
    if per_b:
        out.per_b_hard = [v.value() for v in arrs[0]]
        out.per_b_trivial = [v.value() for v in arrs[1]]
        out.per_b_easy = [v.value() for v in arrs[2]]
    if nseg:
        out.per_seg_hard = [v.value() for v in seg]
    return out


def pi_meissel(x: int, y: int | None = None, c: int = 6) -> int:
    """pi(x) = phi(x, a) + a - 1 - P2, phi by eq. (4.1), y = icbrt(x) by default."""
    if y is None:
        y = icbrt(x)
    return lib().or_pi_meissel(x, y, c)


def s1_p2(x: int, y: int, c: int = 6) -> Decomp:
    """S1 and P2 (with their term counts) of one (x, y, c); the leaf fields
    are zero."""
    D = _Decomp()
    if lib().or_s1_p2(x, y, c, C.byref(D)) != 0:
        raise ValueError(f"or_s1_p2({x}, {y}, {c}) failed")
    vals = {f: getattr(D, f) for f, _ in _Decomp._fields_}
    for k in ("s1", "s2t", "s2e", "s2h", "p2", "phi"):
        vals[k] = vals[k].value()
    return Decomp(**vals)


def leaf_sample(x: int, y: int, c: int, b_lo: int, b_hi: int, u_max: int,
                b_step: int = 1) -> Decomp:
    """The special leaves with b = b_lo + k b_step < b_hi (hard ones only up
    to u_max): a bounded slice of one (x, y, c), for timing the oracle on
    large x or summing it slice by slice."""
    D = _Decomp()
    rc = lib().or_leaf_sample(x, y, c, b_lo, b_hi, b_step, u_max, C.byref(D))
    if rc != 0:
        raise ValueError(f"or_leaf_sample failed with code {rc}")
    vals = {f: getattr(D, f) for f, _ in _Decomp._fields_}
    for k in ("s1", "s2t", "s2e", "s2h", "p2", "phi"):
        vals[k] = vals[k].value()
    return Decomp(**vals)
