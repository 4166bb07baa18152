"""Workgroup-per-shot layout, the autotuner and latency sessions against the
CPU oracle (same bar as the wavefront layout: identical decisions, flags and
iteration counts; FP32 posterior within 1e-5 relative; int8 bit-exact)."""
import os
import tempfile
import time

import numpy as np
import pytest

from workload import bits, lp, noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi  # noqa: E402

from gpu_util import assert_parity, gpu_decode, oracle_decode, to_dev  # noqa: E402

_codes = {}


def code(L):
    if L not in _codes:
        c = lp.lp_code(L)
        _codes[L] = (c, c.hz.dense(), Decoder(c.hz))
    return _codes[L]


def case(L, shots, p, fmt=0, seed=31, per_bit=False, nw=16, max_iters=32, early_stop=True, syn=None,
         layout=abi.QLDPC_LAYOUT_BLOCK):
    c, H, dec = code(L)
    b = noise.Batch(c.hz, seed, np.arange(shots), p)
    s = b.s if syn is None else syn
    if fmt == 0:
        prior = b.gamma
        if per_bit:
            j = noise.rng.uniform(seed, noise.rng.DOMAIN_PRIOR, np.arange(shots)[:, None], np.arange(c.n)[None, :])
            prior = (b.prior_bits() * (0.5 + j)).astype(np.float32)
        scale = prior if per_bit else b.gamma[:, None]
    else:
        prior = b.gamma_q4()
        if per_bit:
            prior = np.repeat(prior[:, None], c.n, axis=1)
        scale = None
    g = gpu_decode(dec, s, prior, fmt=fmt, max_iters=max_iters, early_stop=early_stop, per_bit=per_bit,
                   layout=layout, waves_per_shot=nw)
    o = oracle_decode(H, s, prior, fmt=fmt, max_iters=max_iters, early_stop=early_stop)
    assert_parity(g, o, scale, fmt, tag=f"block L={L} fmt={fmt} nw={nw} pb={per_bit}")
    return g, o


@pytest.mark.parametrize("L", [64, 128])
@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("nw", [8, 16])
def test_block_layout_parity(L, fmt, nw):
    case(L, 48, 0.05, fmt=fmt, nw=nw)


@pytest.mark.parametrize("fmt", [0, 1])
def test_block_layout_per_bit_and_fixed_iterations(fmt):
    case(64, 24, 0.04, fmt=fmt, per_bit=True, seed=32)
    case(64, 24, 0.05, fmt=fmt, max_iters=10, early_stop=False, seed=33)
    g, _ = case(128, 8, 0.05, fmt=fmt, max_iters=1, seed=34)
    assert np.all(g[2] == 1)


def test_block_layout_zero_syndrome():
    c, H, dec = code(64)
    g, _ = case(64, 4, 0.03, syn=np.zeros((4, c.hz.m), np.uint8))
    assert np.all(g[2] == 1) and np.all(g[1] == 1)


def test_block_layout_rejected_for_layered_and_small_lifts():
    for L, sched in ((64, 1), (32, 0)):
        c, H, dec = code(L)
        p = dec.params(sched=sched, layout=abi.QLDPC_LAYOUT_BLOCK)
        err, conv, it, _ = dec.outputs(2)
        with pytest.raises(abi.QldpcError) as ei:
            abi.qldpc_decode_batch(dec.handle, p, 2, torch.zeros((2, dec.syn_words), dtype=torch.int32, device="cuda"),
                                   torch.ones(2, device="cuda"), err, conv, it)
        assert ei.value.status == abi.QLDPC_ERR_UNSUPPORTED


def test_auto_layout_small_batch_parity():
    # AUTO picks the workgroup layout for small flooding batches
    case(64, 3, 0.05, layout=abi.QLDPC_LAYOUT_AUTO, nw=0, seed=35)


def test_autotune_records_a_valid_choice_and_roundtrips():
    c, H, dec = code(64)
    b = noise.Batch(c.hz, 36, np.arange(256), 0.03)
    syn = to_dev(bits.pack_bits(b.s).view(np.int32))
    pr = to_dev(b.gamma)
    err, conv, it, _ = dec.outputs(256)
    p = dec.params()
    best = abi.qldpc_autotune(dec.handle, p, 256, syn, pr, err, conv, it)
    assert best.layout in (abi.QLDPC_LAYOUT_WAVE, abi.QLDPC_LAYOUT_BLOCK, abi.QLDPC_LAYOUT_WAVE_REG)
    assert best.waves_per_shot in (0, 8, 16)
    g = gpu_decode(dec, b.s, b.gamma, layout=0)    # AUTO now uses the recorded choice
    o = oracle_decode(H, b.s, b.gamma)
    assert_parity(g, o, b.gamma[:, None], 0, tag="autotuned")
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "tune.json")
        abi.qldpc_tune_save(dec.handle, f)
        txt = open(f).read()
        assert '"L": 64' in txt and "entries" in txt
        dec2 = Decoder(c.hz)
        abi.qldpc_tune_load(dec2.handle, f)
        abi.qldpc_tune_save(dec2.handle, f + "2")
        assert open(f + "2").read() == txt
        dec2.close()


@pytest.mark.parametrize("io_mode", [abi.QLDPC_IO_COPY, abi.QLDPC_IO_MAPPED, abi.QLDPC_IO_RESIDENT])
@pytest.mark.parametrize("fmt", [0, 1])
def test_session_decode_matches_oracle(io_mode, fmt):
    c, H, dec = code(64)
    b = noise.Batch(c.hz, 37 + fmt, np.arange(80), 0.05)
    prior = b.gamma if fmt == 0 else b.gamma_q4()
    p = dec.params(fmt=fmt)
    s = abi.qldpc_session_create(dec.handle, p, 64, io_mode)
    try:
        syn = np.ascontiguousarray(bits.pack_bits(b.s))
        o = oracle_decode(H, b.s, prior, fmt=fmt)
        for lo, hi in ((0, 1), (1, 65), (65, 80)):
            B = hi - lo
            err = np.zeros((B, dec.err_words), np.uint32)
            conv = np.zeros(B, np.uint8)
            it = np.zeros(B, np.uint8)
            abi.qldpc_session_decode(s, B, syn[lo:hi], np.ascontiguousarray(prior[lo:hi]), err, conv, it)
            e = bits.unpack_bits(err, c.n)
            assert np.array_equal(e, o.e[lo:hi]) and np.array_equal(conv, o.converged[lo:hi])
            assert np.array_equal(it.astype(np.int32), o.iters[lo:hi])
        lat = abi.qldpc_session_latency(s, 50, 1, 80, syn, np.ascontiguousarray(prior))
        assert np.all(lat > 0) and np.isfinite(lat).all()
        print(f"io_mode={io_mode} fmt={fmt} latency p50 {np.percentile(lat, 50):.1f} us "
              f"p99 {np.percentile(lat, 99):.1f} us")
    finally:
        abi.qldpc_session_destroy(s)


@pytest.mark.parametrize("L,fmt,nw,per_bit", [(64, 1, 8, False), (128, 0, 16, True)])
def test_resident_session_survives_idle_exit(L, fmt, nw, per_bit):
    """The resident grid leaves after 200 ms without a request and the next
    request relaunches it; answers before and after equal the oracle's."""
    c, H, dec = code(L)
    n = 12
    b = noise.Batch(c.hz, 41 + L, np.arange(n), 0.05)
    if fmt == 0:
        prior = b.gamma
        if per_bit:
            j = noise.rng.uniform(41, noise.rng.DOMAIN_PRIOR, np.arange(n)[:, None], np.arange(c.n)[None, :])
            prior = (b.prior_bits() * (0.5 + j)).astype(np.float32)
    else:
        prior = b.gamma_q4()
    prior = np.ascontiguousarray(prior)
    syn = np.ascontiguousarray(bits.pack_bits(b.s))
    o = oracle_decode(H, b.s, prior, fmt=fmt)
    s = abi.qldpc_session_create(dec.handle, dec.params(fmt=fmt, per_bit=per_bit, waves_per_shot=nw), 8,
                                 abi.QLDPC_IO_RESIDENT)
    try:
        for k, (lo, hi) in enumerate(((0, 8), (8, 9), (9, 12), (0, 8))):
            if k == 2:
                time.sleep(0.6)      # longer than the idle time: the grid has left
            B = hi - lo
            err = np.zeros((B, dec.err_words), np.uint32)
            conv = np.full(B, 7, np.uint8)
            it = np.zeros(B, np.uint8)
            abi.qldpc_session_decode(s, B, syn[lo:hi], prior[lo:hi], err, conv, it)
            assert np.array_equal(bits.unpack_bits(err, c.n), o.e[lo:hi]), (k, lo, hi)
            assert np.array_equal(conv, o.converged[lo:hi]) and np.array_equal(it.astype(np.int32), o.iters[lo:hi])
    finally:
        abi.qldpc_session_destroy(s)


def test_resident_session_rejects_unsupported_configs():
    for L, kw, mb, status in ((64, dict(sched=abi.QLDPC_LAYERED), 4, abi.QLDPC_ERR_UNSUPPORTED),
                              (32, {}, 4, abi.QLDPC_ERR_UNSUPPORTED),
                              (64, {}, 65, abi.QLDPC_ERR_INVALID_ARG)):
        c, H, dec = code(L)
        with pytest.raises(abi.QldpcError) as ei:
            abi.qldpc_session_create(dec.handle, dec.params(**kw), mb, abi.QLDPC_IO_RESIDENT)
        assert ei.value.status == status, (L, kw, mb)


@pytest.mark.parametrize("fmt", [0, 1])
def test_auto_layout_at_L128_large_batch(fmt):
    """AUTO at L = 128 flooding with a large batch takes the two-wavefront
    register layout and asks for no workspace; it equals that layout and the
    8-wave workgroup layout bit for bit, and a sample of the batch equals the
    oracle."""
    c, H, dec = code(128)
    B = 600
    b = noise.Batch(c.hz, 77 + fmt, np.arange(B), 0.05)
    prior = b.gamma if fmt == 0 else b.gamma_q4()
    assert abi.qldpc_decode_workspace_bytes(dec.handle, dec.params(fmt=fmt), B) == 0
    g_auto = gpu_decode(dec, b.s, prior, fmt=fmt, layout=abi.QLDPC_LAYOUT_AUTO)
    g_reg = gpu_decode(dec, b.s, prior, fmt=fmt, layout=abi.QLDPC_LAYOUT_WAVE_REG)
    g_blk = gpu_decode(dec, b.s, prior, fmt=fmt, layout=abi.QLDPC_LAYOUT_BLOCK, waves_per_shot=8)
    for x, y, z in zip(g_auto, g_reg, g_blk):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    idx = np.arange(0, B, 7)
    o = oracle_decode(H, b.s[idx], prior[idx], fmt=fmt)
    sub = tuple(x[idx] for x in g_auto)
    assert_parity(sub, o, b.gamma[idx][:, None] if fmt == 0 else None, fmt, tag=f"AUTO L=128 fmt={fmt}")
