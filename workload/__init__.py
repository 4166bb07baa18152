"""Seeded synthetic workloads for syndrome decoding of lifted-product codes.

This package generates inputs only (codes, error patterns, syndromes,
priors) and evaluates outcomes (GF(2) logical failures).  It holds none of
the decoder's arithmetic, so the CPU oracle and the device library can both
consume its outputs without sharing any decoding code.
"""
from . import bits, gf2, lp, noise, rng  # noqa: F401
from .lp import LPCode, Side, lp_code, side_from_dense  # noqa: F401
