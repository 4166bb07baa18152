"""Neural min-sum: per-edge, per-iteration weights in place of alpha.

``NeuralMinSum`` is a torch.autograd.Function whose forward and backward are
the library's hand-written kernels (qldpc_nbp_forward / qldpc_nbp_backward):
torch only holds the tensors and runs the optimiser.  The loss is the binary
cross-entropy between the true error bits and sigma(-Q) -- the posterior
probability that a bit flipped -- averaged over iterations, shots and bits:

    L = mean_{k,b,n} [ e softplus(Q) + (1 - e) softplus(-Q) ].

Untrained weights are all alpha, so the untrained decoder is plain
normalized min-sum (Section 2, Algorithm 1).
"""
from __future__ import annotations

import hashlib
import json

import numpy as np

from . import abi


def code_fingerprint(side) -> str:
    """Hash of the lift size and base exponent table (identifies the weights' code)."""
    h = hashlib.sha256()
    h.update(np.int64(side.lift).tobytes())
    h.update(np.ascontiguousarray(side.base, dtype=np.int64).tobytes())
    return h.hexdigest()[:16]


class NeuralMinSum:
    """Namespace for the autograd Function (built lazily so torch is optional
    at import time)."""

    _fn = None

    @classmethod
    def apply(cls, dec, weights, syndromes, priors):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(weights, syndromes, priors, dec)


def _make_function():
    import torch

    class _NMS(torch.autograd.Function):
        @staticmethod
        def forward(ctx, weights, syndromes, priors, dec):
            T = int(weights.shape[0])
            B = int(syndromes.shape[0])
            w = weights.detach().contiguous()
            ws = torch.empty(abi.qldpc_nbp_workspace_bytes(dec.handle, B, T), dtype=torch.uint8,
                             device=weights.device)
            post = torch.empty((T, B, dec.n), dtype=torch.float32, device=weights.device)
            abi.qldpc_nbp_forward(dec.handle, B, T, w, syndromes, priors, post, ws)
            ctx.save_for_backward(w, syndromes, ws)
            ctx.dec = dec
            return post

        @staticmethod
        def backward(ctx, grad_post):
            w, syndromes, ws = ctx.saved_tensors
            T, B = int(w.shape[0]), int(syndromes.shape[0])
            gw = torch.empty_like(w)
            abi.qldpc_nbp_backward(ctx.dec.handle, B, T, w, syndromes, ws, grad_post.contiguous(), gw)
            return gw, None, None, None

    return _NMS


def bce_loss(post, e_true):
    """post [T, B, n] float, e_true [B, n] float 0/1."""
    import torch.nn.functional as F
    e = e_true.unsqueeze(0)
    return (e * F.softplus(post) + (1.0 - e) * F.softplus(-post)).mean()


def init_weights(T: int, nnz: int, alpha: float = 0.75, device="cuda"):
    import torch
    return torch.full((T, nnz), float(alpha), dtype=torch.float32, device=device)


def save_weights(path: str, weights, side, meta: dict | None = None, optimizer=None) -> None:
    """Weights (and optionally optimiser state) keyed by the code fingerprint."""
    import torch
    blob = {"fingerprint": code_fingerprint(side), "weights": weights.detach().cpu(),
            "meta": json.dumps(meta or {})}
    if optimizer is not None:
        blob["optimizer"] = optimizer.state_dict()
    torch.save(blob, path)


def load_weights(path: str, side, device="cuda"):
    import torch
    blob = torch.load(path, map_location="cpu", weights_only=True)
    if blob["fingerprint"] != code_fingerprint(side):
        raise ValueError("weights were trained for a different code")
    return blob["weights"].to(device), json.loads(blob["meta"]), blob.get("optimizer")
