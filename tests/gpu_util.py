"""Helpers for the GPU parity tests: run the C-ABI decoder on workload
batches and compare with the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import oracle
from workload import bits, noise


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_decode(dec, s_bits, prior, fmt=0, sched=0, alpha=0.75, max_iters=32, early_stop=True,
               per_bit=False, posterior=True, layout=0, waves_per_shot=0):
    """Decode uint8 syndrome bits [B, m] on the device; returns host arrays."""
    import torch
    syn = to_dev(bits.pack_bits(s_bits).view(np.int32))
    pr = to_dev(np.asarray(prior, {0: np.float32, 1: np.int8, 2: np.int16}[fmt]))
    p = dec.params(fmt=fmt, sched=sched, alpha=alpha, max_iters=max_iters, early_stop=early_stop,
                   per_bit=per_bit, layout=layout, waves_per_shot=waves_per_shot)
    err, conv, it, post = dec.decode(syn, pr, p, posterior=posterior)
    torch.cuda.synchronize()
    e = bits.unpack_bits(err.cpu().numpy().view(np.uint32), dec.n)
    return (e, conv.cpu().numpy(), it.cpu().numpy().astype(np.int32),
            None if post is None else post.cpu().numpy())


def oracle_decode(H, s_bits, prior, fmt=0, sched=0, alpha=0.75, max_iters=32, early_stop=True,
                  layer_size=None):
    if fmt == 0 and sched == 0:
        return oracle.flood_f32(H, s_bits, prior, alpha=alpha, max_iters=max_iters, early_stop=early_stop)
    if fmt == 1 and sched == 0:
        return oracle.flood_i8(H, s_bits, prior, alpha=alpha, max_iters=max_iters, early_stop=early_stop)
    if fmt == 2 and sched == 0:
        return oracle.flood_i16(H, s_bits, prior, alpha=alpha, max_iters=max_iters, early_stop=early_stop)
    if fmt == 2:
        return oracle.layered_i16(H, s_bits, prior, layer_size, alpha=alpha, max_iters=max_iters,
                                  early_stop=early_stop)
    if fmt == 0 and sched == 1:
        return oracle.layered_f32(H, s_bits, prior, layer_size, alpha=alpha, max_iters=max_iters,
                                  early_stop=early_stop)
    return oracle.layered_i8(H, s_bits, prior, layer_size, alpha=alpha, max_iters=max_iters,
                             early_stop=early_stop)


def assert_parity(g, o, prior_scale, fmt, tag=""):
    """Identical e / converged / iterations; posterior within 1e-5 relative
    (FP32: |dQ| <= 1e-5 * max(|Q_oracle|, |gamma|)), bit-exact for int8 and
    int16."""
    e, conv, it, post = g
    bad = np.nonzero(~np.all(e == o.e, axis=1) | (conv != o.converged) | (it != o.iters))[0]
    assert bad.size == 0, (f"{tag}: {bad.size} shots differ, first {bad[:8].tolist()}; "
                           f"gpu iters {it[bad[:4]].tolist()} oracle {o.iters[bad[:4]].tolist()}")
    if post is not None:
        if fmt != 0:
            assert np.array_equal(post, o.Q), f"{tag}: integer posterior not bit-exact"
        else:
            tol = 1e-5 * np.maximum(np.abs(o.Q), np.abs(prior_scale))
            d = np.abs(post - o.Q)
            assert np.all(d <= tol), f"{tag}: max posterior error {float((d - tol).max())}"
