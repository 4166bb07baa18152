"""int16 saturating messages with Q8 priors (QLDPC_I16Q8) against the CPU
oracle, bit-exact: hard decisions, convergence flags, iteration counts and
posteriors (Q / 256), in every layout, lift and block pattern, including a
saturation-heavy case where most messages sit at the +-32767 bound."""
import numpy as np
import pytest

from workload import bits, lp, noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi  # noqa: E402

from gpu_util import assert_parity, gpu_decode, oracle_decode  # noqa: E402

I16 = abi.QLDPC_I16Q8
WAVE, BLOCK, REG, HBM = (abi.QLDPC_LAYOUT_WAVE, abi.QLDPC_LAYOUT_BLOCK, abi.QLDPC_LAYOUT_WAVE_REG,
                         abi.QLDPC_LAYOUT_HBM)
_sides = {}


def side(L, which=0):
    if (L, which) not in _sides:
        c = lp.lp_code(L)
        sd = c.hx if which else c.hz
        _sides[(L, which)] = (sd, sd.dense(), Decoder(sd))
    return _sides[(L, which)]


def q8_priors(b, seed, per_bit, n):
    q = b.gamma_q8()
    if not per_bit:
        return q
    j = noise.rng.uniform(seed, noise.rng.DOMAIN_PRIOR, np.arange(b.B)[:, None], np.arange(n)[None, :])
    return np.clip(np.round(q[:, None] * (0.5 + j)), -32767, 32767).astype(np.int16)


def case(L, shots, p, layout, sched=0, per_bit=False, which=0, seed=301, max_iters=32, early_stop=True,
         alpha=0.75, nw=0, prior=None, syn=None):
    sd, H, dec = side(L, which)
    b = noise.Batch(sd, seed, np.arange(shots), p)
    s = b.s if syn is None else syn
    pr = q8_priors(b, seed, per_bit, sd.n) if prior is None else prior
    g = gpu_decode(dec, s, pr, fmt=I16, sched=sched, alpha=alpha, max_iters=max_iters, early_stop=early_stop,
                   per_bit=per_bit or pr.ndim == 2, layout=layout, waves_per_shot=nw)
    o = oracle_decode(H, s, pr, fmt=I16, sched=sched, alpha=alpha, max_iters=max_iters, early_stop=early_stop,
                      layer_size=L)
    assert_parity(g, o, None, I16, tag=f"int16 L={L} layout={layout} sched={sched} pb={per_bit} which={which}")
    return g, o


def test_q8_quantiser_matches_the_workload_definition():
    llr = np.array([4.59512, 3.476099, 2.944439, -2.5, 0.0, 1000.0, -1000.0, 0.001953125], np.float32)
    assert np.array_equal(abi.qldpc_quantize_prior_q8(llr), noise.quantize_q8(llr))
    assert noise.quantize_q8(np.float32(np.log(0.97 / 0.03)))[()] == 890


@pytest.mark.parametrize("L", [16, 32, 64])
@pytest.mark.parametrize("sched", [0, 1])
def test_register_layout(L, sched):
    case(L, 300 if L < 64 else 130, 0.05, REG, sched=sched, seed=311)          # ragged last wave
    case(L, 90, 0.03, REG, sched=sched, per_bit=True, seed=312)


@pytest.mark.parametrize("L", [16, 32, 64, 128])
@pytest.mark.parametrize("sched", [0, 1])
def test_lds_layout_all_lifts(L, sched):
    case(L, 67, 0.05, WAVE, sched=sched, seed=313)
    case(L, 33, 0.04, WAVE, sched=sched, per_bit=True, seed=314)


@pytest.mark.parametrize("L", [64, 128])
@pytest.mark.parametrize("nw", [8, 16])
def test_workgroup_layout(L, nw):
    case(L, 40, 0.05, BLOCK, nw=nw, seed=315)
    case(L, 24, 0.04, BLOCK, nw=nw, per_bit=True, seed=316)


@pytest.mark.parametrize("L", [128, 256])
def test_hbm_layout(L):
    case(L, 24, 0.05, HBM, seed=317)
    case(L, 12, 0.04, HBM, per_bit=True, max_iters=6, early_stop=False, seed=318)


@pytest.mark.parametrize("layout,L", [(REG, 64), (WAVE, 64), (BLOCK, 64), (WAVE, 128), (HBM, 128)])
def test_hx_pattern(layout, L):
    case(L, 48, 0.05, layout, which=1, seed=319)
    if layout in (REG, WAVE):
        case(L, 48, 0.05, layout, which=1, sched=1, seed=320)


@pytest.mark.parametrize("layout", [REG, WAVE, BLOCK])
def test_saturation_heavy_priors(layout):
    """Per-bit priors spread over the whole int16 range: most messages are
    formed at the saturation bound, so a wrong bound or an int8-width
    intermediate changes decisions and posteriors."""
    L, shots = 64, 40
    sd, H, dec = side(L)
    u = noise.rng.uniform(321, noise.rng.DOMAIN_PRIOR, np.arange(shots)[:, None], np.arange(sd.n)[None, :])
    prior = np.round((u - 0.3) * 2 * 32767).clip(-32767, 32767).astype(np.int16)
    g, o = case(L, shots, 0.05, layout, prior=prior, max_iters=8, early_stop=False, seed=321)
    assert np.abs(o.Q).max() * 256 > 32767       # posteriors beyond the message range were reached
    case(L, shots, 0.05, layout, sched=0, prior=prior, seed=322)


@pytest.mark.parametrize("layout", [REG, WAVE])
def test_fixed_iterations_alpha_and_zero_syndrome(layout):
    case(64, 64, 0.05, layout, max_iters=10, early_stop=False, seed=323)
    g, _ = case(64, 37, 0.05, layout, max_iters=1, seed=324)
    assert np.all(g[2] == 1)
    case(32, 64, 0.05, layout, alpha=1.0, seed=325)
    case(32, 64, 0.05, layout, alpha=0.5, sched=1, seed=326)
    sd, H, dec = side(64)
    g, _ = case(64, 3, 0.03, layout, syn=np.zeros((3, sd.m), np.uint8), seed=327)
    assert np.all(g[2] == 1) and np.all(g[1] == 1) and not g[0].any()


def test_resident_session():
    L = 64
    sd, H, dec = side(L)
    b = noise.Batch(sd, 328, np.arange(20), 0.05)
    prior = np.ascontiguousarray(b.gamma_q8())
    syn = np.ascontiguousarray(bits.pack_bits(b.s))
    o = oracle_decode(H, b.s, prior, fmt=I16)
    s = abi.qldpc_session_create(dec.handle, dec.params(fmt=I16, waves_per_shot=16), 16, abi.QLDPC_IO_RESIDENT)
    try:
        for lo, hi in ((0, 1), (1, 17), (17, 20)):
            B = hi - lo
            err = np.zeros((B, dec.err_words), np.uint32)
            conv = np.full(B, 7, np.uint8)
            it = np.zeros(B, np.uint8)
            abi.qldpc_session_decode(s, B, syn[lo:hi], prior[lo:hi], err, conv, it)
            assert np.array_equal(bits.unpack_bits(err, sd.n), o.e[lo:hi])
            assert np.array_equal(conv, o.converged[lo:hi]) and np.array_equal(it.astype(np.int32), o.iters[lo:hi])
    finally:
        abi.qldpc_session_destroy(s)


def test_workspace_bytes_and_auto_layout():
    sd, H, dec = side(256)
    hbm = abi.QLDPC_LAYOUT_HBM
    assert abi.qldpc_decode_workspace_bytes(dec.handle, dec.params(fmt=I16, layout=hbm), 8) == 8 * 120 * 256 * 2
    assert abi.qldpc_decode_workspace_bytes(dec.handle, dec.params(fmt=I16), 8) == 0     # AUTO: registers
    sd64, H64, dec64 = side(64)
    assert abi.qldpc_decode_workspace_bytes(dec64.handle, dec64.params(fmt=I16), 8) == 0
    case(64, 100, 0.05, 0, seed=329)                       # AUTO at L = 64
    with pytest.raises(abi.QldpcError) as ei:
        p = dec64.params(fmt=I16, alpha=0.7)                # not num / 2^s
        abi.qldpc_decode_batch(dec64.handle, p, 1, torch.zeros((1, dec64.syn_words), dtype=torch.int32,
                                                               device="cuda"),
                               torch.ones(1, dtype=torch.int16, device="cuda"), *dec64.outputs(1)[:3], None)
    assert ei.value.status == abi.QLDPC_ERR_UNSUPPORTED


@pytest.mark.parametrize("sched", [0, 1])
def test_full_batch_sampled(sched):
    """65536 shots at L = 64 in the register layout, the launch the benchmark
    times: every converged shot reproduces its syndrome, and a sample
    (every 2048th shot, the last, and unconverged ones) equals the oracle."""
    L, B = 64, 65536
    sd, H, dec = side(L)
    b = noise.Batch(sd, 1400 + sched, np.arange(B), 0.05)
    prior = b.gamma_q8()
    e, conv, it, _ = gpu_decode(dec, b.s, prior, fmt=I16, sched=sched, posterior=False, layout=REG)
    ok = conv == 1
    assert ok.mean() > 0.5
    assert np.array_equal(noise.syndromes(sd, e[ok]), b.s[ok])
    idx = np.unique(np.concatenate([np.arange(0, B, 2048), [B - 1], np.nonzero(~ok)[0][:6]]))
    o = oracle_decode(H, b.s[idx], prior[idx], fmt=I16, sched=sched, layer_size=L)
    assert np.array_equal(e[idx], o.e) and np.array_equal(conv[idx], o.converged)
    assert np.array_equal(it[idx], o.iters)
