"""Seeded synthetic query sets for pi(x) (inputs only: no arithmetic of the
method).  The paper's workloads are single values of x (Tables 1-3); these
are the many-query mixes used to measure batching and serving."""
from __future__ import annotations

import numpy as np


def log_uniform_x(n: int, lo_exp: float, hi_exp: float, seed: int) -> list[int]:
    """x_i = floor(10^e_i), e_i uniform in [lo_exp, hi_exp), PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.uniform(lo_exp, hi_exp, n)
    return [int(np.floor(10.0 ** v)) for v in e]


def batch_queries(n: int = 4096, seed: int = 1503) -> list[int]:
    """The batch mix: x log-uniform in [1e8, 1e15]."""
    return log_uniform_x(n, 8.0, 15.0, seed)


def serve_stream(n: int = 20000, rate_per_s: float = 100.0, lo_exp: float = 10.0,
                 hi_exp: float = 18.0, seed: int = 1839) -> tuple[list[int], list[float]]:
    """An open-loop Poisson arrival stream: x log-uniform in [1e10, 1e18] and
    arrival times (seconds from the start) with exponential gaps of mean
    1 / rate_per_s, both from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.uniform(lo_exp, hi_exp, n)
    gaps = rng.exponential(1.0 / rate_per_s, n)
    xs = [int(np.floor(10.0 ** v)) for v in e]
    return xs, list(np.cumsum(gaps))
