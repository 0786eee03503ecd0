"""Seeded synthetic inputs for the benchmark and the parity tests.

Holds none of the method's arithmetic: only the input recipes.  All draws use
numpy's PCG64 generator; values are drawn in FP64 and rounded (RNE) to the
storage dtype.  The default seed is the one the paper quotes for its
benchmark angles (Section 4).
"""
from __future__ import annotations

import math

import numpy as np

SEED = 2024873


def _rng(seed: int | None):
    return np.random.default_rng(SEED if seed is None else seed)


def uniform(n: int, lo: float, hi: float, seed: int | None = None,
            dtype=np.float32) -> np.ndarray:
    """n values U[lo, hi], drawn in FP64, rounded to `dtype`."""
    return _rng(seed).uniform(lo, hi, n).astype(dtype)


def small_uniform(n: int = 1 << 20, seed: int | None = None) -> np.ndarray:
    """2^20 FP32 angles, U[-2 pi, 2 pi]."""
    return uniform(n, -2 * math.pi, 2 * math.pi, seed)


def throughput_mix(n: int = 1 << 28, seed: int | None = None,
                   chunk: int = 1 << 24) -> np.ndarray:
    """99% U[-1000, 1000]; 1% within 1e-3 of an odd multiple of pi/2,
    (2m+1) pi/2 + U[-1e-3, 1e-3] with m uniform in [-318, 317] (|x| < 998).
    Positions are random.  FP32."""
    rng = _rng(seed)
    out = np.empty(n, np.float32)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        x = rng.uniform(-1000.0, 1000.0, m)
        pole = rng.random(m) < 0.01
        k = int(pole.sum())
        mm = rng.integers(-318, 318, k).astype(np.float64)
        x[pole] = (2 * mm + 1) * (math.pi / 2) + rng.uniform(-1e-3, 1e-3, k)
        out[s:s + m] = x.astype(np.float32)
    return out


def half_precision_uniform(n: int, kind: str, seed: int | None = None):
    """U[-pi, pi] rounded to FP16 (kind 'f16') or BF16 (kind 'bf16').
    Returns raw 16-bit patterns as uint16."""
    x = _rng(seed).uniform(-math.pi, math.pi, n)
    return round_to_16(x, kind)


def log_magnitude(n: int = 1 << 26, seed: int | None = None) -> np.ndarray:
    """|x| = 10^U[0, 6], random sign: large arguments for the reduction
    (q up to ~6.4e5), all below the 2^29 bit-table threshold.  FP32."""
    rng = _rng(seed)
    mag = 10.0 ** rng.uniform(0.0, 6.0, n)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return (sign * mag).astype(np.float32)


def protocol_f64(n: int = 1 << 27, seed: int | None = None,
                 chunk: int = 1 << 24) -> np.ndarray:
    """The paper's benchmark angles (Section 4): U[-1e6, 1e6] in FP64."""
    rng = _rng(seed)
    out = np.empty(n, np.float64)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        out[s:s + m] = rng.uniform(-1e6, 1e6, m)
    return out


def log_magnitude_f64(n: int, seed: int | None = None) -> np.ndarray:
    """|x| = 10^U[-300, 300], random sign: every FP64 exponent range, most
    of it through the large-|x| reduction.  FP64."""
    rng = _rng(seed)
    mag = 10.0 ** rng.uniform(-300.0, 300.0, n)
    return np.where(rng.random(n) < 0.5, -mag, mag)


def exponent_sweep_f64(per_exp: int = 16, seed: int | None = None):
    """per_exp random significands at every binary exponent of FP64 (normal
    and subnormal), both signs."""
    rng = _rng(seed)
    e = np.repeat(np.arange(-1074, 1024), per_exp)
    x = np.ldexp(1.0 + rng.random(e.size), e)
    return np.where(rng.random(e.size) < 0.5, -x, x)


def normal_pair(shape, sigma_x: float, seed: int | None = None):
    """x ~ N(0, sigma_x^2), upstream gradient g ~ N(0, 1); FP32."""
    rng = _rng(seed)
    n = int(np.prod(shape))
    x = (rng.standard_normal(n) * sigma_x).astype(np.float32).reshape(shape)
    g = rng.standard_normal(n).astype(np.float32).reshape(shape)
    return x, g


# ---------------------------------------------------------------------------
# 16-bit patterns (storage only)
# ---------------------------------------------------------------------------

def round_to_16(x: np.ndarray, kind: str) -> np.ndarray:
    """Round FP64 values to FP16 or BF16 (nearest, ties to even); returns the
    raw uint16 patterns."""
    x = np.asarray(x, np.float64)
    if kind == "f16":
        # beyond the FP16 range the nearest-even result is +-Inf
        with np.errstate(over="ignore"):
            return x.astype(np.float16).view(np.uint16)
    if kind != "bf16":
        raise ValueError(kind)
    # BF16 = top half of FP32: round FP64 -> BF16 directly (no double
    # rounding through FP32).
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    ee = np.maximum(e, -125)                 # BF16 subnormal grid 2^-133
    q = np.ldexp(np.rint(np.ldexp(x, 8 - ee)), ee - 8)
    with np.errstate(over="ignore"):
        f = q.astype(np.float32)             # exact: q has <= 8 bits
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def all_16bit_patterns() -> np.ndarray:
    return np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)


def decode_16(u: np.ndarray, kind: str) -> np.ndarray:
    """Raw uint16 patterns -> FP64 values (exact)."""
    u = np.asarray(u, np.uint16)
    if kind == "f16":
        return u.view(np.float16).astype(np.float64)
    # signalling-NaN patterns raise numpy's "invalid" flag when widened (they
    # come out as quiet NaNs); every other pattern widens exactly
    with np.errstate(invalid="ignore"):
        return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
