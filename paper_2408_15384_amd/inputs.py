"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module draws numbers and shapes only; it holds none of the
product's arithmetic.

Distributions (all from ``numpy.random.default_rng(seed)``; A is drawn before
B):

* ``uniform_f64``  -- entries uniform on [-1, 1) in binary64 (2*U - 1, exact).
* ``uniform_f32``  -- the same drawn natively in FP32 (2*U - 1 is exact in FP32
  for the 24-bit grid ``Generator.random`` returns, so no entry reaches 1.0).
* ``integer``      -- integers uniform on [lo, hi] (default [-8, 8]) stored as
  floating point; every product and partial sum of such inputs is exact.
* ``m2e_f32``      -- m * 2**e with m uniform over the FP32 grid of [1, 2) and
  e a uniform integer in [-8, 8]; all entries positive.
* ``box_muller``   -- N(0, 1) entries by the Box-Muller transform (paper
  section IV), with U1 drawn from (0, 1] so the logarithm stays finite.
* ``log_uniform_dims`` -- round(exp(U(ln lo, ln hi))) clamped to [lo, hi].
* ``poisson_arrivals`` -- cumulative exponential gaps at a fixed rate.
"""
from __future__ import annotations

import numpy as np


def rng_for(seed) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_f64(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.random(shape, dtype=np.float64) * 2.0 - 1.0


def uniform_f32(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.random(shape, dtype=np.float32) * np.float32(2.0) - np.float32(1.0)


def integer(rng: np.random.Generator, shape, dtype=np.float64, lo: int = -8, hi: int = 8) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=shape).astype(dtype)


def m2e_f32(rng: np.random.Generator, shape, emin: int = -8, emax: int = 8) -> np.ndarray:
    frac = rng.integers(0, 1 << 23, size=shape, dtype=np.uint32)
    m = (np.uint32(0x3F800000) | frac).view(np.float32)
    e = rng.integers(emin, emax + 1, size=shape)
    return (m * np.exp2(e).astype(np.float32)).astype(np.float32)


def box_muller(rng: np.random.Generator, shape) -> np.ndarray:
    n = int(np.prod(shape))
    half = (n + 1) // 2
    u1 = 1.0 - rng.random(half)          # (0, 1]
    u2 = rng.random(half)
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * half)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:n].reshape(shape)


def pair(kind: str, M: int, N: int, K: int, seed=0):
    """(A, B) of the named distribution: A is M x K, B is K x N, A drawn first."""
    rng = rng_for(seed)
    if kind == "uniform_f64":
        return uniform_f64(rng, (M, K)), uniform_f64(rng, (K, N))
    if kind == "uniform_f32":
        return uniform_f32(rng, (M, K)), uniform_f32(rng, (K, N))
    if kind == "int_f64":
        return integer(rng, (M, K)), integer(rng, (K, N))
    if kind == "int_f32":
        return integer(rng, (M, K), np.float32), integer(rng, (K, N), np.float32)
    if kind == "m2e_f32":
        return m2e_f32(rng, (M, K)), m2e_f32(rng, (K, N))
    if kind == "normal_f64":
        return box_muller(rng, (M, K)), box_muller(rng, (K, N))
    raise ValueError(f"unknown input kind {kind!r}")


def log_uniform_dims(rng: np.random.Generator, count: int, lo: int, hi: int) -> np.ndarray:
    v = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count)))
    return np.clip(v, lo, hi).astype(np.int64)


def grouped_shapes(count: int = 512, lo: int = 32, hi: int = 1024, seed=0) -> np.ndarray:
    """(count, 3) array of (M, N, K), each dimension log-uniform on [lo, hi]."""
    rng = rng_for(seed)
    return log_uniform_dims(rng, 3 * count, lo, hi).reshape(count, 3)


def poisson_arrivals(rng: np.random.Generator, count: int, rate: float) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def serving_requests(count: int = 10000, rate: float = 20000.0, lo: int = 64, hi: int = 4096,
                     frac_f64: float = 0.5, seed=0):
    """Request stream: arrival times (s), (M, N, K) and an is_f64 flag each."""
    rng = rng_for(seed)
    t = poisson_arrivals(rng, count, rate)
    dims = log_uniform_dims(rng, 3 * count, lo, hi).reshape(count, 3)
    is_f64 = rng.random(count) < frac_f64
    return t, dims, is_f64


def probe_vector(n: int, seed=0) -> np.ndarray:
    """Residual-probe vector: binary64 entries uniform on [-1, 1)."""
    return uniform_f64(rng_for([0x9E37, int(seed)]), (n,))
