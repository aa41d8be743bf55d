"""Seeded synthetic inputs shared by the tests and the benchmark.

This module only draws random numbers and shapes them into series; it holds
none of the DTW method's arithmetic.  Every generator is seeded from
``numpy.random.Generator(PCG64)``; all generation is in float64 and the values
the GPU reads are the float32 rounding of them (``as_f32``), which the oracle
reads back promoted to float64 (``as_oracle``), so both sides see identical
numbers.

Workloads (the paper measures on six real datasets that are not available;
these seeded generators stand in for them with the paper's query lengths and
window ratios):

* ``c1``  one random-walk query of length 128 against a 20,000-point
  random-walk series, window 13 (10 %).
* ``c2``  noisy multi-sinusoid (3 periods in [16, 512], SNR 10 dB), a
  2,000,000-point series and a length-256 query cut from an independent
  realisation plus N(0, 0.1) noise; windows {0, 13, 26, 52}.
* ``c3``  2,000 standardised random walks of length 512, full window.
* ``c4``  64 random-walk queries with lengths uniform in [64, 1024] and window
  ratios uniform in [0.05, 0.20] against a 10,000,000-point random walk.
* ``c5``  4,096 pairs of standardised random walks of length 256, the second a
  randomly time-warped copy of the first plus N(0, 0.2) noise, window 26.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2010_05371


def rng(config: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, config, sub])))


def as_f32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def as_oracle(x32) -> np.ndarray:
    return np.asarray(x32, dtype=np.float32).astype(np.float64)


def window_from_ratio(ratio: float, m: int) -> int:
    """Integer Sakoe-Chiba window from a ratio of the query length (rounded up)."""
    return int(math.ceil(ratio * m - 1e-9))


def random_walk(n: int, g: np.random.Generator) -> np.ndarray:
    return np.cumsum(g.standard_normal(n))


def standardise(x: np.ndarray) -> np.ndarray:
    """Zero mean, unit (population) standard deviation: part of the input recipe."""
    x = np.asarray(x, dtype=np.float64)
    return (x - x.mean()) / x.std()


def multi_sinusoid(n: int, periods, phases, g: np.random.Generator, snr_db: float = 10.0):
    t = np.arange(n, dtype=np.float64)
    s = np.zeros(n)
    for P, phi in zip(periods, phases):
        s += np.sin(2.0 * np.pi * t / P + phi)
    noise_var = np.mean(s * s) / (10.0 ** (snr_db / 10.0))
    return s + g.normal(0.0, math.sqrt(noise_var), n)


def warped_copy(S: np.ndarray, g: np.random.Generator, warp_sd: float = 0.5,
                noise_sd: float = 0.2) -> np.ndarray:
    """Monotone random time warp phi of [0, L-1] onto itself, T = S(phi) + noise."""
    L = S.size
    inc = np.exp(g.normal(0.0, warp_sd, L - 1))
    phi = np.concatenate([[0.0], np.cumsum(inc)])
    phi *= (L - 1) / phi[-1]
    return np.interp(phi, np.arange(L, dtype=np.float64), S) + g.normal(0.0, noise_sd, L)


# --------------------------------------------------------------------------- workloads

def c1(n: int = 20_000, m: int = 128):
    g = rng(1)
    query = random_walk(m, g)
    series = random_walk(n, rng(1, 1))
    return as_f32(query), as_f32(series), window_from_ratio(0.10, m)


C2_WINDOWS = (0, 13, 26, 52)  # 0 %, 5 %, 10 %, 20 % of 256, rounded up


def c2(n: int = 2_000_000, m: int = 256):
    g = rng(2)
    periods = g.uniform(16.0, 512.0, 3)
    series = multi_sinusoid(n, periods, g.uniform(0.0, 2.0 * np.pi, 3), rng(2, 1))
    g2 = rng(2, 2)
    indep = multi_sinusoid(4 * m, periods, g2.uniform(0.0, 2.0 * np.pi, 3), g2)
    off = int(g2.integers(0, 3 * m))
    query = indep[off:off + m] + g2.normal(0.0, 0.1, m)
    return as_f32(query), as_f32(series), [window_from_ratio(f, m) for f in (0.0, 0.05, 0.10, 0.20)]


def erp_pairs(base: int = 4096, reps: int = 64, L: int = 256):
    """ERP pair batch: `base` pairs of a z-normalised random walk and a warped
    noisy copy of it, the whole set repeated `reps` times (row p is pair
    p mod base); float32 [base*reps, L] each."""
    g = rng(7300)
    X = np.stack([standardise(random_walk(L, g)) for _ in range(base)])
    Y = np.stack([warped_copy(x, g) for x in X])
    return np.tile(as_f32(X), (reps, 1)), np.tile(as_f32(Y), (reps, 1))


def c3(N: int = 2000, L: int = 512):
    g = rng(3)
    X = np.stack([standardise(random_walk(L, g)) for _ in range(N)])
    return as_f32(X), L - 1


def c4(nq: int = 64, n: int = 10_000_000, mlo: int = 64, mhi: int = 1024):
    g = rng(4)
    ms = g.integers(mlo, mhi + 1, nq)
    ratios = g.uniform(0.05, 0.20, nq)
    queries = [as_f32(random_walk(int(m), g)) for m in ms]
    windows = [window_from_ratio(float(rt), int(m)) for rt, m in zip(ratios, ms)]
    series = as_f32(random_walk(n, rng(4, 1)))
    return queries, windows, series


def c5(P: int = 4096, L: int = 256):
    g = rng(5)
    S = np.empty((P, L))
    T = np.empty((P, L))
    for p in range(P):
        s = standardise(random_walk(L, g))
        S[p] = s
        T[p] = standardise(warped_copy(s, g))
    return as_f32(S), as_f32(T), window_from_ratio(0.10, L)


def random_pairs(P: int, L: int, seed: int, scale: float = 1.0):
    """Independent standardised random-walk pairs for parity tests."""
    g = rng(100, seed)
    S = np.stack([standardise(random_walk(L, g)) for _ in range(P)]) * scale
    T = np.stack([standardise(random_walk(L, g)) for _ in range(P)]) * scale
    return as_f32(S), as_f32(T)


def plant(series: np.ndarray, query: np.ndarray, offset: int, a: float = 1.0,
          b: float = 0.0) -> np.ndarray:
    """Copy of `series` with a*query+b written at `offset` (an exact z-normalised match)."""
    x = np.array(series, dtype=np.float64)
    x[offset:offset + query.size] = a * np.asarray(query, dtype=np.float64) + b
    return as_f32(x)
