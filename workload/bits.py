"""Bit packing used at the library boundary.

Bit i of a vector lives in bit (i mod 32) of 32-bit word floor(i / 32),
least significant bit first; rows are padded to whole words with zeros.
"""
from __future__ import annotations

import numpy as np


def words(nbits: int) -> int:
    return (nbits + 31) // 32


def pack_bits(b: np.ndarray) -> np.ndarray:
    """uint8 0/1 [B, n] -> uint32 [B, ceil(n/32)]."""
    b = np.asarray(b, dtype=np.uint8)
    B, n = b.shape
    w = words(n)
    pad = np.zeros((B, w * 32), dtype=np.uint8)
    pad[:, :n] = b & 1
    by = np.packbits(pad.reshape(B, w * 4, 8), axis=2, bitorder="little").reshape(B, w * 4)
    return by.view("<u4").reshape(B, w).astype(np.uint32)


def unpack_bits(words_: np.ndarray, n: int) -> np.ndarray:
    """uint32 [B, w] -> uint8 0/1 [B, n]."""
    w = np.ascontiguousarray(np.asarray(words_, dtype=np.uint32))
    B = w.shape[0]
    by = w.astype("<u4").view(np.uint8).reshape(B, -1)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return bits[:, :n].copy()
