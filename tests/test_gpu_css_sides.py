"""Both sides of the CSS code: the H_X block pattern decodes like H_Z, against
the oracle, in every layout (register-resident, LDS wavefront, workgroup,
resident session), and one mixed batch holding H_Z and H_X shots of the same
codes decodes every shot exactly as it decodes alone (the paper decodes the
two sides together, Section 2)."""
import numpy as np
import pytest

from workload import bits, lp, noise
from workload.mixed import MixedBatch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi  # noqa: E402

from gpu_util import assert_parity, gpu_decode, oracle_decode, to_dev  # noqa: E402

WAVE, BLOCK, REG = abi.QLDPC_LAYOUT_WAVE, abi.QLDPC_LAYOUT_BLOCK, abi.QLDPC_LAYOUT_WAVE_REG
_sides = {}


def side(L, which):
    if (L, which) not in _sides:
        c = lp.lp_code(L)
        sd = c.hx if which else c.hz
        _sides[(L, which)] = (c, sd, sd.dense(), Decoder(sd))
    return _sides[(L, which)]


def test_css_condition_and_shapes():
    for L in (16, 64):
        c, hx, Hx, _ = side(L, 1)
        _, hz, Hz, _ = side(L, 0)
        assert hx.m == hz.m and hx.n == hz.n and hx.nnz == hz.nnz
        assert not np.any((Hx.astype(np.int64) @ Hz.T.astype(np.int64)) % 2)
        assert not np.array_equal(Hx, Hz)


@pytest.mark.parametrize("L,layout,fmt", [(16, REG, 0), (32, REG, 0), (64, REG, 0), (16, WAVE, 1), (64, WAVE, 0),
                                          (64, WAVE, 1), (128, WAVE, 0), (128, WAVE, 1), (64, BLOCK, 0),
                                          (64, BLOCK, 1), (128, BLOCK, 0), (128, REG, 0), (128, REG, 1)])
def test_hx_side_matches_oracle(L, layout, fmt):
    c, sd, H, dec = side(L, 1)
    b = noise.Batch(sd, 61 + L + fmt, np.arange(150 if L < 128 else 60), 0.05)
    prior = b.gamma if fmt == 0 else b.gamma_q4()
    g = gpu_decode(dec, b.s, prior, fmt=fmt, layout=layout)
    o = oracle_decode(H, b.s, prior, fmt=fmt)
    assert_parity(g, o, b.gamma[:, None] if fmt == 0 else None, fmt, tag=f"H_X L={L} layout={layout} fmt={fmt}")
    ok = g[1] == 1
    assert np.array_equal(noise.syndromes(sd, g[0][ok]), b.s[ok])


@pytest.mark.parametrize("fmt", [0, 1])
def test_hx_side_layered(fmt):
    c, sd, H, dec = side(64, 1)
    b = noise.Batch(sd, 71 + fmt, np.arange(120), 0.05)
    prior = b.gamma if fmt == 0 else b.gamma_q4()
    g = gpu_decode(dec, b.s, prior, fmt=fmt, sched=1, layout=WAVE)
    o = oracle_decode(H, b.s, prior, fmt=fmt, sched=1, layer_size=64)
    assert_parity(g, o, b.gamma[:, None] if fmt == 0 else None, fmt, tag=f"H_X layered fmt={fmt}")


def test_hx_resident_session():
    c, sd, H, dec = side(64, 1)
    b = noise.Batch(sd, 81, np.arange(20), 0.05)
    syn = np.ascontiguousarray(bits.pack_bits(b.s))
    pr = np.ascontiguousarray(b.gamma)
    o = oracle_decode(H, b.s, pr)
    s = abi.qldpc_session_create(dec.handle, dec.params(), 8, abi.QLDPC_IO_RESIDENT)
    try:
        for lo, hi in ((0, 8), (8, 9), (9, 17)):
            B = hi - lo
            err = np.zeros((B, dec.err_words), np.uint32)
            conv = np.zeros(B, np.uint8)
            it = np.zeros(B, np.uint8)
            abi.qldpc_session_decode(s, B, syn[lo:hi], pr[lo:hi], err, conv, it)
            assert np.array_equal(bits.unpack_bits(err, sd.n), o.e[lo:hi])
            assert np.array_equal(conv, o.converged[lo:hi]) and np.array_equal(it.astype(np.int32), o.iters[lo:hi])
    finally:
        abi.qldpc_session_destroy(s)


def test_mixed_batch_decodes_both_sides_together():
    """H_Z and H_X of the L = 64 code, H_X of L = 16 and L = 128 in one
    batch: every shot equals its single-code decode."""
    keys = [(64, 0), (64, 1), (16, 1), (128, 1)]
    sides = [side(L, w) for L, w in keys]
    mb = MixedBatch([s_[0] for s_ in sides], 91, 3000, sides=[s_[1] for s_ in sides])
    decs = [s_[3] for s_ in sides]
    prm = decs[0].params(max_iters=32)
    plan = abi.qldpc_mixed_create([d.handle for d in decs], prm, mb.B, True)
    try:
        dev = [to_dev(mb.cid.astype(np.int32)), to_dev(mb.syn_off), to_dev(mb.err_off),
               to_dev(mb.syn.view(np.int32)), to_dev(mb.gamma)]
        err = torch.full((mb.err_words,), -1, dtype=torch.int32, device="cuda")
        conv = torch.full((mb.B,), 7, dtype=torch.uint8, device="cuda")
        it = torch.zeros(mb.B, dtype=torch.uint8, device="cuda")
        abi.qldpc_mixed_decode(plan, mb.B, *dev, err, conv, it)
        torch.cuda.synchronize()
        e_all = mb.split_errors(err.cpu().numpy().view(np.uint32))
        conv_h, it_h = conv.cpu().numpy(), it.cpu().numpy().astype(np.int32)
    finally:
        abi.qldpc_mixed_destroy(plan)
    for c, (L, w) in enumerate(keys):
        idx, _ = mb.e[c]
        assert idx.size > 0, (L, w)
        g = gpu_decode(decs[c], mb.s[c], mb.gamma[idx], posterior=False)
        assert np.array_equal(e_all[c], g[0]), (L, w)
        assert np.array_equal(conv_h[idx], g[1]) and np.array_equal(it_h[idx], g[2]), (L, w)


@pytest.mark.parametrize("L,fmt,nw", [(64, 0, 16), (64, 1, 8), (128, 0, 16)])
def test_css_pair_resident_session(L, fmt, nw):
    """One request decodes both sides of a CSS code: the H_Z syndrome of X
    errors and the H_X syndrome of independent Z errors, each against the
    oracle on its own parity-check matrix, for one pair and for several."""
    c, hz, Hz, dz = side(L, 0)
    _, hx, Hx, dx = side(L, 1)
    n = 20
    bz = noise.Batch(hz, 501 + L, np.arange(n), 0.05)
    bx = noise.Batch(hx, 601 + L, np.arange(n), 0.03)
    pz = bz.gamma if fmt == 0 else bz.gamma_q4()
    px = bx.gamma if fmt == 0 else bx.gamma_q4()
    oz = oracle_decode(Hz, bz.s, pz, fmt=fmt)
    ox = oracle_decode(Hx, bx.s, px, fmt=fmt)
    # pairs: [n][2][...], H_Z side first
    syn = np.ascontiguousarray(np.stack([bits.pack_bits(bz.s), bits.pack_bits(bx.s)], axis=1).reshape(2 * n, -1))
    prior = np.ascontiguousarray(np.stack([pz, px], axis=1).reshape(2 * n))
    s = abi.qldpc_session_create_css(dz.handle, dx.handle, dz.params(fmt=fmt, waves_per_shot=nw), 8)
    try:
        for lo, hi in ((0, 1), (1, 9), (9, 12), (12, 20)):
            B = hi - lo
            err = np.zeros((2 * B, dz.err_words), np.uint32)
            conv = np.full(2 * B, 7, np.uint8)
            it = np.zeros(2 * B, np.uint8)
            abi.qldpc_session_decode(s, B, syn[2 * lo:2 * hi], prior[2 * lo:2 * hi], err, conv, it)
            e = bits.unpack_bits(err, hz.n)
            assert np.array_equal(e[0::2], oz.e[lo:hi]) and np.array_equal(e[1::2], ox.e[lo:hi]), (lo, hi)
            assert np.array_equal(conv[0::2], oz.converged[lo:hi]) and np.array_equal(conv[1::2], ox.converged[lo:hi])
            assert np.array_equal(it[0::2].astype(np.int32), oz.iters[lo:hi])
            assert np.array_equal(it[1::2].astype(np.int32), ox.iters[lo:hi])
        lat = abi.qldpc_session_latency(s, 200, 1, n, syn, prior)
        assert np.all(lat > 0) and np.isfinite(lat).all()
    finally:
        abi.qldpc_session_destroy(s)


def test_css_pair_session_rejects_bad_pairs():
    c, hz, Hz, dz = side(64, 0)
    _, hx, Hx, dx = side(64, 1)
    _, hx128, _, dx128 = side(128, 1)
    for a_, b_, kw, mp in ((dx, dz, {}, 4), (dz, dx128, {}, 4), (dz, dx, {}, 33), (dz, dx, {}, 0),
                           (dz, dx, dict(fmt=abi.QLDPC_I16Q8), 4)):
        with pytest.raises(abi.QldpcError) as ei:
            abi.qldpc_session_create_css(a_.handle, b_.handle, dz.params(**kw), mp)
        assert ei.value.status in (abi.QLDPC_ERR_INVALID_ARG, abi.QLDPC_ERR_UNSUPPORTED)
    s = abi.qldpc_session_create_css(dz.handle, dx.handle, dz.params(), 2)
    try:
        with pytest.raises(abi.QldpcError) as ei:      # 3 pairs > max_pairs
            abi.qldpc_session_decode(s, 3, np.zeros((6, dz.syn_words), np.uint32), np.ones(6, np.float32),
                                     np.zeros((6, dz.err_words), np.uint32), np.zeros(6, np.uint8),
                                     np.zeros(6, np.uint8))
        assert ei.value.status == abi.QLDPC_ERR_INVALID_ARG
    finally:
        abi.qldpc_session_destroy(s)
