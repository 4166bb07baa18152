"""MI355X syndrome min-sum decoder for quantum LDPC codes.

Normalized min-sum for syndrome-based decoding (Section 2, Algorithm 1) of
quasi-cyclic lifted-product CSS codes, as hand-written HIP kernels behind
the C ABI in include/qldpc.h.  ``abi`` mirrors the C functions one to one;
``Decoder`` is a convenience wrapper that owns a code object and allocates
output tensors with torch.  Nothing here computes a decoding step.
"""
from __future__ import annotations

from . import abi
from .abi import QldpcError  # noqa: F401

__all__ = ["abi", "Decoder", "QldpcError"]


class Decoder:
    """One CSS side (an LP code's H_Z or H_X) resident on one device."""

    def __init__(self, side, device: int = 0):
        self.m, self.n = int(side.m), int(side.n)
        self.handle = abi.qldpc_code_create(side.m, side.n, side.row_ptr, side.col_idx,
                                            side.lift, side.base, device)
        self.device = device
        _, _, self.nnz, self.max_dc, self.max_dv = abi.qldpc_code_info(self.handle)

    def close(self):
        if self.handle is not None:
            abi.qldpc_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def syn_words(self) -> int:
        return (self.m + 31) // 32

    @property
    def err_words(self) -> int:
        return (self.n + 31) // 32

    def params(self, fmt=abi.QLDPC_F32, sched=abi.QLDPC_FLOOD, alpha=0.75, max_iters=32,
               early_stop=True, per_bit=False, layout=abi.QLDPC_LAYOUT_AUTO, waves_per_shot=0):
        p = abi.qldpc_default_params()
        p.fmt, p.sched, p.alpha, p.max_iters = int(fmt), int(sched), float(alpha), int(max_iters)
        p.early_stop = int(bool(early_stop))
        p.prior_mode = abi.QLDPC_PRIOR_PER_BIT if per_bit else abi.QLDPC_PRIOR_PER_SHOT
        p.layout = int(layout)
        p.waves_per_shot = int(waves_per_shot)
        return p

    def outputs(self, batch: int, posterior: bool = False):
        import torch
        dev = torch.device("cuda", self.device)
        err = torch.empty((batch, self.err_words), dtype=torch.int32, device=dev)
        conv = torch.empty((batch,), dtype=torch.uint8, device=dev)
        it = torch.empty((batch,), dtype=torch.uint8, device=dev)
        post = torch.empty((batch, self.n), dtype=torch.float32, device=dev) if posterior else None
        return err, conv, it, post

    def decode(self, syndromes, priors, params=None, posterior: bool = False, out=None, stream=None):
        """syndromes: int32 [B, ceil(m/32)] packed; priors: float32, int8 or int16,
        [B] or [B, n].  Returns (errors int32 [B, ceil(n/32)], converged u8,
        iterations u8, posterior or None)."""
        params = params or self.params()
        B = int(syndromes.shape[0])
        err, conv, it, post = out if out is not None else self.outputs(B, posterior)
        need = abi.qldpc_decode_workspace_bytes(self.handle, params, B)
        if need == 0:
            abi.qldpc_decode_batch(self.handle, params, B, syndromes, priors, err, conv, it, post, stream)
        else:
            # messages in device memory (large lifts): a workspace from torch's allocator
            import torch
            ws = torch.empty(need + 256, dtype=torch.uint8, device=err.device)
            base = ws.data_ptr()
            off = (-base) % 256
            abi.qldpc_decode_batch_ws(self.handle, params, B, syndromes, priors, err, conv, it, post,
                                      base + off, need, stream)
            self._ws = ws   # keep it alive until the next decode on this object
        return err, conv, it, post
