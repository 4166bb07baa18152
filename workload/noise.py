"""Seeded synthetic decoding inputs: error patterns, syndromes and priors.

Noise model (code capacity, X side): each qubit flips independently with
probability p, e_n = [u(seed, shot, n) < p].  The syndrome the decoder sees
is s = H_Z e^T over GF(2) (Section 2).  The per-bit prior of normalized
min-sum is the log-likelihood ratio gamma = log((1 - p) / p), rounded once to
float32.  The int8 format carries priors as signed Q4 fixed point:
round-half-away-from-zero(16 * gamma) clamped to [-127, 127]; the int16
format as signed Q8: round-half-away-from-zero(256 * gamma) clamped to
[-32767, 32767].

Nothing here decodes; these are inputs shared by the oracle and the device
path.
"""
from __future__ import annotations

import numpy as np

from . import rng
from .bits import pack_bits


def _workers() -> int:
    import os
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def errors(seed: int, shots, n: int, p, chunk: int = 1024) -> np.ndarray:
    """uint8 [len(shots), n] Bernoulli(p) error bits; p scalar or per shot.

    Row blocks are drawn on a few threads (numpy releases the interpreter
    lock in its array loops); each value depends only on (seed, shot, bit)."""
    shots = np.asarray(shots, dtype=np.int64)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), shots.shape)
    out = np.empty((shots.size, n), dtype=np.uint8)

    def block(lo):
        hi = min(lo + chunk, shots.size)
        u = rng.uniform_rows(seed, rng.DOMAIN_ERROR, shots[lo:hi], n, chunk=chunk)
        out[lo:hi] = u < p[lo:hi, None]

    starts = range(0, shots.size, chunk)
    if shots.size <= chunk:
        for lo in starts:
            block(lo)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(block, starts))
    return out


def syndromes(side, e: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """uint8 [B, m] syndrome bits s = H e^T mod 2 (row-wise XOR over CSR)."""
    B = e.shape[0]
    s = np.zeros((B, side.m), dtype=np.uint8)
    deg = np.diff(side.row_ptr)

    def block(lo):
        blk = e[lo:lo + chunk]
        if np.all(deg == deg[0]):
            g = blk[:, side.col_idx].reshape(blk.shape[0], side.m, int(deg[0]))
            s[lo:lo + chunk] = np.bitwise_xor.reduce(g, axis=2)
        else:
            for r in range(side.m):
                cols = side.col_idx[side.row_ptr[r]:side.row_ptr[r + 1]]
                s[lo:lo + chunk, r] = np.bitwise_xor.reduce(blk[:, cols], axis=1) if cols.size else 0

    starts = range(0, B, chunk)
    if B <= chunk:
        for lo in starts:
            block(lo)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(block, starts))
    return s


def random_syndromes(seed: int, shots, m: int) -> np.ndarray:
    """uint8 [len(shots), m] uniformly random syndrome bits."""
    u = rng.uniform_rows(seed, rng.DOMAIN_SYNDROME, np.asarray(shots), m)
    return (u < 0.5).astype(np.uint8)


def llr(p) -> np.ndarray:
    """float32 log((1-p)/p), computed in float64 and rounded once."""
    p = np.asarray(p, dtype=np.float64)
    return np.log((1.0 - p) / p).astype(np.float32)


def quantize_q4(gamma) -> np.ndarray:
    """int8 Q4 prior: clamp(round-half-away(16 * gamma), -127, 127).

    16 * gamma is exact in float32, so the only rounding is the final one.
    """
    g = np.asarray(gamma, dtype=np.float32) * np.float32(16.0)
    r = np.sign(g) * np.floor(np.abs(g).astype(np.float64) + 0.5)
    return np.clip(r, -127, 127).astype(np.int8)


def quantize_q8(gamma) -> np.ndarray:
    """int16 Q8 prior: clamp(round-half-away(256 * gamma), -32767, 32767).

    256 * gamma is exact in float32, so the only rounding is the final one.
    """
    g = np.asarray(gamma, dtype=np.float32) * np.float32(256.0)
    r = np.sign(g) * np.floor(np.abs(g).astype(np.float64) + 0.5)
    return np.clip(r, -32767, 32767).astype(np.int16)


def shot_rates(seed: int, shots, lo: float = 0.01, hi: float = 0.08) -> np.ndarray:
    """Per-shot noise rate p ~ U[lo, hi)."""
    u = rng.uniform(seed, rng.DOMAIN_PSHOT, np.asarray(shots), 0)
    return lo + (hi - lo) * u


def code_mix(seed: int, nshots: int, ncodes: int):
    """Dirichlet(1,..,1) proportions, then a per-shot categorical code id.

    Dirichlet(1,...,1) is sampled as normalised Exp(1) draws.
    Returns (proportions float64 [ncodes], code id int32 [nshots]).
    """
    g = -np.log(1.0 - rng.uniform(seed, rng.DOMAIN_MIX, 0, np.arange(ncodes)))
    prop = g / g.sum()
    u = rng.uniform(seed, rng.DOMAIN_MIX, 1, np.arange(nshots))
    cid = np.searchsorted(np.cumsum(prop), u, side="right")
    return prop, np.minimum(cid, ncodes - 1).astype(np.int32)


class Batch:
    """One decoding batch on one side of a code, all arrays host-resident."""

    def __init__(self, side, seed: int, shots, p):
        shots = np.asarray(shots, dtype=np.int64)
        self.side = side
        self.seed = seed
        self.shots = shots
        self.p = np.broadcast_to(np.asarray(p, dtype=np.float64), shots.shape).copy()
        self.e = errors(seed, shots, side.n, self.p)
        self.s = syndromes(side, self.e)
        self.gamma = llr(self.p)                 # float32 [B] per-shot prior

    @property
    def B(self) -> int:
        return int(self.shots.size)

    def s_packed(self) -> np.ndarray:
        return pack_bits(self.s)

    def gamma_q4(self) -> np.ndarray:
        return quantize_q4(self.gamma)

    def gamma_q8(self) -> np.ndarray:
        return quantize_q8(self.gamma)

    def prior_bits(self) -> np.ndarray:
        """float32 [B, n]: the per-shot prior broadcast to every bit."""
        return np.repeat(self.gamma[:, None], self.side.n, axis=1)
