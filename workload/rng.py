"""Counter-based random numbers for the synthetic workloads.

Every random quantity in a workload (code exponents, error patterns, per-shot
noise rates, code mixes) is a pure function of ``(seed, domain, a, b)``.  A
value can therefore be regenerated for one shot without replaying a stream,
and any language can reproduce it.

The mixing function is SplitMix64's finaliser (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014):

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

applied to ``x + GAMMA`` with GAMMA = 0x9E3779B97F4A7C15 (the golden-ratio
increment of the same paper).  Keys are chained:

    k1   = mix(seed + GAMMA * (domain + 1))
    k2   = mix(k1   + GAMMA * (a + 1))
    draw = mix(k2   + GAMMA * (b + 1))

and a uniform double is ``(draw >> 11) * 2**-53``.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Domains keep independent uses of one seed apart.
DOMAIN_CODE = 1      # LP base exponents
DOMAIN_ERROR = 2     # Bernoulli error bits
DOMAIN_PSHOT = 3     # per-shot noise rate
DOMAIN_MIX = 4       # code proportions and per-shot code choice
DOMAIN_SYNDROME = 5  # uniformly random (usually inconsistent) syndromes
DOMAIN_PRIOR = 6     # per-bit prior jitter


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _step(key: np.ndarray, c) -> np.ndarray:
    c = np.asarray(c, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + GAMMA * (c + np.uint64(1)))


def key(seed: int, domain: int, a=0) -> np.ndarray:
    """Second-level key for ``(seed, domain, a)``; ``a`` may be an array."""
    k1 = _step(np.uint64(seed & 0xFFFFFFFFFFFFFFFF), domain)
    return _step(k1, a)


def draws(seed: int, domain: int, a, b) -> np.ndarray:
    """Raw 64-bit draws, broadcasting ``a`` against ``b``."""
    k2 = key(seed, domain, a)
    return _step(k2, b)


def uniform(seed: int, domain: int, a, b) -> np.ndarray:
    """Uniform doubles in [0, 1)."""
    d = draws(seed, domain, a, b)
    return (d >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_rows(seed: int, domain: int, rows: np.ndarray, ncols: int,
                 chunk: int = 4096) -> np.ndarray:
    """Uniform doubles, shape [len(rows), ncols], row r uses a = rows[r]."""
    rows = np.asarray(rows, dtype=np.uint64)
    out = np.empty((rows.size, ncols), dtype=np.float64)
    cols = np.arange(ncols, dtype=np.uint64)[None, :]
    for s in range(0, rows.size, chunk):
        k2 = key(seed, domain, rows[s:s + chunk])[:, None]
        out[s:s + chunk] = (_step(k2, cols) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return out
