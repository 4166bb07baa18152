"""Uneven mixed batches: shots of several lifted codes with per-shot noise
rates, laid out as ragged packed buffers (one syndrome row and one error row
per shot, each of that shot's code width, concatenated)."""
from __future__ import annotations

import numpy as np

from . import bits, noise


class MixedBatch:
    def __init__(self, codes, seed: int, nshots: int, p_lo: float = 0.01, p_hi: float = 0.08, sides=None):
        """codes: list of LPCode; shot i has code cid[i] (Dirichlet(1,..)
        proportions then a categorical draw) and rate p[i] ~ U[p_lo, p_hi).
        sides: the parity-check side decoded for each code (default: H_Z of
        every code; H_X of a code gives syndromes of its Z errors)."""
        self.codes = codes
        self.sides = list(sides) if sides is not None else [c.hz for c in codes]
        self.prop, self.cid = noise.code_mix(seed, nshots, len(codes))
        self.p = noise.shot_rates(seed, np.arange(nshots), p_lo, p_hi)
        self.gamma = noise.llr(self.p)
        self.B = nshots
        sw = np.array([(sd.m + 31) // 32 for sd in self.sides])
        ew = np.array([(sd.n + 31) // 32 for sd in self.sides])
        self.syn_off = np.concatenate([[0], np.cumsum(sw[self.cid])[:-1]]).astype(np.int64)
        self.err_off = np.concatenate([[0], np.cumsum(ew[self.cid])[:-1]]).astype(np.int64)
        self.syn_words = int(sw[self.cid].sum())
        self.err_words = int(ew[self.cid].sum())
        self.syn = np.zeros(self.syn_words, np.uint32)
        self.e = {}     # code index -> (shot indices, error bits [k, n])
        self.s = {}     # code index -> syndrome bits [k, m]
        for c, sd in enumerate(self.sides):
            idx = np.nonzero(self.cid == c)[0]
            e = noise.errors(seed, idx, sd.n, self.p[idx])
            s = noise.syndromes(sd, e)
            self.e[c] = (idx, e)
            self.s[c] = s
            pk = bits.pack_bits(s)
            if idx.size:
                pos = self.syn_off[idx][:, None] + np.arange(sw[c])[None, :]
                self.syn[pos] = pk

    def split_errors(self, err_words: np.ndarray):
        """Per code: decision bits [k, n] of that code's shots, in shot order."""
        out = {}
        for c, sd in enumerate(self.sides):
            idx = self.e[c][0]
            ew = (sd.n + 31) // 32
            rows = err_words[self.err_off[idx][:, None] + np.arange(ew)[None, :]] if idx.size else \
                np.zeros((0, ew), np.uint32)
            out[c] = bits.unpack_bits(rows, sd.n)
        return out
