"""Device decoder (through the C ABI) against the CPU oracle.

The bar: identical hard decisions, convergence flags and iteration counts
per shot; FP32 posteriors within 1e-5 relative error
(|dQ| <= 1e-5 * max(|Q_oracle|, |gamma|)); int8 posteriors bit-exact.
Inputs are the seeded workloads: lifted-product codes LP(A, A*) with a 3x5
monomial base, iid X flips, H_Z syndromes.
"""
import numpy as np
import pytest

from workload import lp, noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi  # noqa: E402

from gpu_util import assert_parity, gpu_decode, oracle_decode  # noqa: E402

_codes = {}


def code(L):
    if L not in _codes:
        c = lp.lp_code(L)
        _codes[L] = (c, c.hz.dense(), Decoder(c.hz))
    return _codes[L]


def run_case(L, shots, p, fmt=0, sched=0, per_bit=False, seed=7, max_iters=32, early_stop=True,
             alpha=0.75, syn=None, layout=abi.QLDPC_LAYOUT_WAVE):
    c, H, dec = code(L)
    b = noise.Batch(c.hz, seed, np.arange(shots), p)
    s = b.s if syn is None else syn
    if fmt == 0:
        prior = b.prior_bits() if per_bit else b.gamma
        if per_bit:
            # per-bit jitter so that every bit has its own prior
            j = noise.rng.uniform(seed, noise.rng.DOMAIN_PRIOR, np.arange(shots)[:, None],
                                  np.arange(c.n)[None, :])
            prior = (prior * (0.5 + j)).astype(np.float32)
        scale = prior if per_bit else b.gamma[:, None]
    else:
        q = b.gamma_q4()
        if per_bit:
            j = noise.rng.uniform(seed, noise.rng.DOMAIN_PRIOR, np.arange(shots)[:, None],
                                  np.arange(c.n)[None, :])
            q = np.clip(np.round(q[:, None] * (0.5 + j)), -127, 127).astype(np.int8)
        prior = q
        scale = None
    g = gpu_decode(dec, s, prior, fmt=fmt, sched=sched, max_iters=max_iters, early_stop=early_stop,
                   per_bit=per_bit, alpha=alpha, layout=layout)
    o = oracle_decode(H, s, prior, fmt=fmt, sched=sched, max_iters=max_iters, early_stop=early_stop,
                      layer_size=L, alpha=alpha)
    assert_parity(g, o, scale, fmt, tag=f"L={L} p={p} fmt={fmt} sched={sched} pb={per_bit} layout={layout}")
    return g, o


def test_config0_fp32_flood_1000_shots():
    """L = 16 (N = 544), p = 0.03, alpha 0.75, flooding, 32 iterations, FP32."""
    g, o = run_case(16, 1000, 0.03)
    assert o.converged.mean() > 0.9


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("p", [0.01, 0.03, 0.05])
def test_L64_formats_and_schedules(fmt, sched, p):
    run_case(64, 192, p, fmt=fmt, sched=sched, seed=11)


@pytest.mark.parametrize("L", [16, 32, 64, 128])
@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("sched", [0, 1])
def test_all_lifts(L, fmt, sched):
    # shot counts leave a ragged last wave for L < 64
    run_case(L, 67, 0.05, fmt=fmt, sched=sched, seed=13)


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("L", [16, 64, 128])
def test_per_bit_priors(fmt, L):
    run_case(L, 45, 0.04, fmt=fmt, per_bit=True, seed=17)
    run_case(L, 45, 0.04, fmt=fmt, sched=1, per_bit=True, seed=18)


@pytest.mark.parametrize("fmt", [0, 1])
def test_fixed_iterations_and_one_iteration(fmt):
    run_case(64, 64, 0.05, fmt=fmt, max_iters=10, early_stop=False, seed=19)
    g, o = run_case(64, 64, 0.05, fmt=fmt, max_iters=1, seed=20)
    assert np.all(g[2] == 1)


def test_alpha_one_and_half():
    run_case(32, 64, 0.05, alpha=1.0, seed=21)
    run_case(32, 64, 0.05, fmt=1, alpha=0.5, seed=22)


def test_zero_and_inconsistent_syndromes():
    c, H, dec = code(64)
    z = np.zeros((5, c.hz.m), np.uint8)
    g, o = run_case(64, 5, 0.03, syn=z)
    assert np.all(g[2] == 1) and np.all(g[1] == 1) and not g[0].any()
    rnd = noise.random_syndromes(23, np.arange(40), c.hz.m)
    g, o = run_case(64, 40, 0.03, syn=rnd, max_iters=12)
    # H_Z has rank m - 8 for this code, so almost every random syndrome is
    # inconsistent and can never converge
    assert g[1].sum() <= 2


def test_single_shot_and_empty_batch():
    run_case(64, 1, 0.05, seed=24)
    run_case(16, 1, 0.05, seed=25)
    c, H, dec = code(64)
    err, conv, it, post = dec.outputs(0)
    dec.decode(torch.zeros((0, dec.syn_words), dtype=torch.int32, device="cuda"),
               torch.zeros((0,), dtype=torch.float32, device="cuda"), out=(err, conv, it, post))
    torch.cuda.synchronize()


def test_deterministic_and_order_independent():
    c, H, dec = code(64)
    b = noise.Batch(c.hz, 26, np.arange(128), 0.05)
    W = abi.QLDPC_LAYOUT_WAVE
    g1 = gpu_decode(dec, b.s, b.gamma, layout=W)
    g2 = gpu_decode(dec, b.s, b.gamma, layout=W)
    perm = np.random.default_rng(0).permutation(128)
    g3 = gpu_decode(dec, b.s[perm], b.gamma[perm], layout=W)
    for a_, b_ in zip(g1, g2):
        assert np.array_equal(a_, b_)
    for a_, b_ in zip(g1, g3):
        assert np.array_equal(a_[perm], b_)


def test_invalid_arguments():
    c, H, dec = code(64)
    p = dec.params(max_iters=0)
    err, conv, it, post = dec.outputs(4)
    syn = torch.zeros((4, dec.syn_words), dtype=torch.int32, device="cuda")
    pr = torch.ones(4, dtype=torch.float32, device="cuda")
    with pytest.raises(abi.QldpcError) as ei:
        abi.qldpc_decode_batch(dec.handle, p, 4, syn, pr, err, conv, it, None)
    assert ei.value.status == abi.QLDPC_ERR_INVALID_ARG
    p = dec.params(fmt=abi.QLDPC_I8Q4, alpha=0.7)
    with pytest.raises(abi.QldpcError) as ei:
        abi.qldpc_decode_batch(dec.handle, p, 4, syn, pr, err, conv, it, None)
    assert ei.value.status == abi.QLDPC_ERR_UNSUPPORTED


REG = abi.QLDPC_LAYOUT_WAVE_REG


@pytest.mark.parametrize("L", [16, 32, 64])
@pytest.mark.parametrize("per_bit", [False, True])
def test_register_resident_layout(L, per_bit):
    """Messages in registers, moved between lanes by permutes: the same
    decisions, flags, iteration counts and posteriors as the oracle."""
    run_case(L, 300 if L < 64 else 130, 0.05, per_bit=per_bit, seed=17, layout=REG)
    run_case(L, 200, 0.02, per_bit=per_bit, seed=18, layout=REG)


def test_register_resident_edge_cases():
    run_case(64, 40, 0.05, max_iters=10, early_stop=False, seed=19, layout=REG)
    g, _ = run_case(16, 37, 0.05, max_iters=1, seed=20, layout=REG)          # ragged: 37 = 9 waves + 1 shot
    assert np.all(g[2] == 1)
    run_case(32, 33, 0.04, alpha=1.0, seed=21, layout=REG)                   # ragged: 16 waves + 1 shot
    run_case(64, 50, 0.03, alpha=0.5, seed=22, layout=REG)
    c, H, dec = code(64)
    g, _ = run_case(64, 3, 0.03, syn=np.zeros((3, c.hz.m), np.uint8), seed=23, layout=REG)
    assert np.all(g[1] == 1) and np.all(g[2] == 1)


@pytest.mark.parametrize("L", [16, 32, 64])
@pytest.mark.parametrize("per_bit", [False, True])
def test_register_resident_layered(L, per_bit):
    """Layered schedule with check messages and a-posteriori values in
    registers: identical to the oracle's layered decoder (layer = block row)."""
    run_case(L, 300 if L < 64 else 130, 0.05, sched=1, per_bit=per_bit, seed=27, layout=REG)
    run_case(L, 100, 0.03, sched=1, per_bit=per_bit, max_iters=7, early_stop=False, seed=28, layout=REG)


@pytest.mark.parametrize("L", [16, 64])
@pytest.mark.parametrize("sched", [0, 1])
def test_register_resident_int8_bit_exact(L, sched):
    """int8 messages held as 32-bit integers in registers: bit-exact
    decisions, flags, iterations and posteriors against the int8 oracle."""
    run_case(L, 300 if L < 64 else 130, 0.05, fmt=1, sched=sched, seed=37, layout=REG)
    run_case(L, 120, 0.04, fmt=1, sched=sched, per_bit=True, seed=38, layout=REG)
    run_case(L, 60, 0.05, fmt=1, sched=sched, max_iters=5, early_stop=False, seed=39, layout=REG)


@pytest.mark.parametrize("fmt", [0, 1, 2])
@pytest.mark.parametrize("per_bit", [False, True])
def test_register_resident_L128(fmt, per_bit):
    """L = 128 with messages in registers: one workgroup of two wavefronts per
    shot, each holding half of every circulant's rows, the variable pass and
    the syndrome test exchanging through LDS.  Same decisions, flags,
    iterations and posteriors as the oracle (FP32 within 1e-5, integer
    formats bit-exact)."""
    run_case(128, 96, 0.05, fmt=fmt, per_bit=per_bit, seed=57, layout=REG)
    run_case(128, 64, 0.02, fmt=fmt, per_bit=per_bit, seed=58, layout=REG)


def test_register_resident_L128_edge_cases():
    run_case(128, 40, 0.05, max_iters=10, early_stop=False, seed=59, layout=REG)
    g, _ = run_case(128, 17, 0.05, max_iters=1, seed=60, layout=REG)
    assert np.all(g[2] == 1)
    run_case(128, 33, 0.04, alpha=1.0, seed=61, layout=REG)
    run_case(128, 21, 0.03, alpha=0.5, seed=62, layout=REG)
    c, H, dec = code(128)
    g, _ = run_case(128, 3, 0.03, syn=np.zeros((3, c.hz.m), np.uint8), seed=63, layout=REG)
    assert np.all(g[1] == 1) and np.all(g[2] == 1)
    # the H_X block pattern
    dx = Decoder(c.hx)
    b = noise.Batch(c.hx, 64, np.arange(80), 0.05)
    gx = gpu_decode(dx, b.s, b.gamma, layout=REG)
    ox = oracle_decode(c.hx.dense(), b.s, b.gamma)
    assert_parity(gx, ox, b.gamma[:, None], 0, tag="L=128 H_X register layout")


def test_register_resident_L128_large_batch_sampled():
    """32768 shots at p = 0.05 in one launch: converged shots reproduce their
    syndromes, a sample matches the oracle shot by shot, and every shot
    equals the 8-wave workgroup layout's decode."""
    c, H, dec = code(128)
    B = 32768
    b = noise.Batch(c.hz, 1100, np.arange(B), 0.05)
    g = gpu_decode(dec, b.s, b.gamma, posterior=False, layout=REG)
    gb = gpu_decode(dec, b.s, b.gamma, posterior=False, layout=abi.QLDPC_LAYOUT_BLOCK, waves_per_shot=8)
    for x, y in zip(g[:3], gb[:3]):
        assert np.array_equal(x, y)
    e, conv, it, _ = g
    ok = conv == 1
    assert ok.mean() > 0.5
    assert np.array_equal(noise.syndromes(c.hz, e[ok]), b.s[ok])
    idx = np.unique(np.concatenate([np.arange(0, B, 2048), [B - 1], np.nonzero(~ok)[0][:8]]))
    o = oracle_decode(H, b.s[idx], b.gamma[idx])
    assert np.array_equal(e[idx], o.e) and np.array_equal(conv[idx], o.converged)
    assert np.array_equal(it[idx], o.iters)


@pytest.mark.parametrize("L,fmt,per_bit", [(256, 0, False), (256, 1, False), (256, 2, False), (256, 0, True),
                                             (256, 1, True), (512, 0, False), (512, 1, False), (512, 2, True)])
def test_register_resident_large_lifts(L, fmt, per_bit):
    """L = 256 and 512 with messages in registers: one workgroup of L / 64
    wavefronts per shot.  Same decisions, flags, iterations and posteriors as
    the oracle (FP32 within 1e-5, integer formats bit-exact), and identical
    to the layout with messages in HBM."""
    shots = 40 if L == 256 else 12
    g, _ = run_case(L, shots, 0.05, fmt=fmt, per_bit=per_bit, seed=70 + L // 64 + fmt, layout=REG)
    g_h, _ = run_case(L, shots, 0.05, fmt=fmt, per_bit=per_bit, seed=70 + L // 64 + fmt, layout=abi.QLDPC_LAYOUT_HBM)
    for x, y in zip(g, g_h):
        assert np.array_equal(x, y)


def test_register_resident_large_lift_edge_cases():
    run_case(256, 24, 0.05, max_iters=6, early_stop=False, seed=80, layout=REG)
    g, _ = run_case(256, 9, 0.05, max_iters=1, seed=81, layout=REG)
    assert np.all(g[2] == 1)
    run_case(256, 16, 0.04, alpha=1.0, seed=82, layout=REG)
    c, H, dec = code(256)
    g, _ = run_case(256, 3, 0.03, syn=np.zeros((3, c.hz.m), np.uint8), seed=83, layout=REG)
    assert np.all(g[1] == 1) and np.all(g[2] == 1)
    for L in (256, 512):
        c = lp.lp_code(L)
        dx = Decoder(c.hx)
        b = noise.Batch(c.hx, 84, np.arange(16 if L == 256 else 6), 0.05)
        gx = gpu_decode(dx, b.s, b.gamma, layout=REG)
        ox = oracle_decode(c.hx.dense(), b.s, b.gamma)
        assert_parity(gx, ox, b.gamma[:, None], 0, tag=f"L={L} H_X register layout")


def test_register_resident_L256_large_batch_sampled():
    """8192 shots at p = 0.05 in one launch: every shot equals the HBM
    layout's decode, converged shots reproduce their syndromes, and a sample
    matches the oracle shot by shot."""
    c, H, dec = code(256)
    B = 8192
    b = noise.Batch(c.hz, 1300, np.arange(B), 0.05)
    g = gpu_decode(dec, b.s, b.gamma, posterior=False, layout=REG)
    gh = gpu_decode(dec, b.s, b.gamma, posterior=False, layout=abi.QLDPC_LAYOUT_HBM)
    for x, y in zip(g[:3], gh[:3]):
        assert np.array_equal(x, y)
    e, conv, it, _ = g
    ok = conv == 1
    assert ok.mean() > 0.5
    assert np.array_equal(noise.syndromes(c.hz, e[ok]), b.s[ok])
    idx = np.unique(np.concatenate([np.arange(0, B, 2048), [B - 1], np.nonzero(~ok)[0][:4]]))
    o = oracle_decode(H, b.s[idx], b.gamma[idx])
    assert np.array_equal(e[idx], o.e) and np.array_equal(conv[idx], o.converged)
    assert np.array_equal(it[idx], o.iters)


def test_register_resident_rejects_unsupported():
    for L, fmt, sched in ((128, 0, 1), (128, 1, 1), (256, 0, 1), (512, 1, 1)):
        c, H, dec = code(L)
        p = dec.params(fmt=fmt, sched=sched, layout=REG)
        err, conv, it, _ = dec.outputs(2)
        syn = torch.zeros((2, dec.syn_words), dtype=torch.int32, device="cuda")
        pr = torch.ones(2, device="cuda") if fmt == 0 else torch.ones(2, dtype=torch.int8, device="cuda")
        with pytest.raises(abi.QldpcError) as ei:
            abi.qldpc_decode_batch(dec.handle, p, 2, syn, pr, err, conv, it, None)
        assert ei.value.status == abi.QLDPC_ERR_UNSUPPORTED, (L, fmt, sched)


@pytest.mark.parametrize("fmt,sched,layout", [(0, 0, abi.QLDPC_LAYOUT_WAVE), (1, 0, abi.QLDPC_LAYOUT_WAVE),
                                              (0, 1, abi.QLDPC_LAYOUT_WAVE), (1, 1, abi.QLDPC_LAYOUT_WAVE),
                                              (0, 0, abi.QLDPC_LAYOUT_WAVE_REG), (0, 1, abi.QLDPC_LAYOUT_WAVE_REG),
                                              (1, 0, abi.QLDPC_LAYOUT_WAVE_REG), (1, 1, abi.QLDPC_LAYOUT_WAVE_REG)])
def test_full_batch_sampled(fmt, sched, layout):
    """65536 shots at L = 64, p = 0.05, as the benchmark launches them; the
    oracle re-decodes a sample of shots one by one, and every converged shot
    must reproduce its syndrome."""
    c, H, dec = code(64)
    B = 65536
    b = noise.Batch(c.hz, 1000 + fmt + 2 * sched, np.arange(B), 0.05)
    prior = b.gamma if fmt == 0 else b.gamma_q4()
    g = gpu_decode(dec, b.s, prior, fmt=fmt, sched=sched, posterior=False, layout=layout)
    e, conv, it, _ = g
    ok = conv == 1
    assert np.array_equal(noise.syndromes(c.hz, e[ok]), b.s[ok])
    assert ok.mean() > 0.5
    idx = np.unique(np.concatenate([np.arange(0, B, 1024), [B - 1], np.nonzero(~ok)[0][:16]]))
    o = oracle_decode(H, b.s[idx], prior[idx], fmt=fmt, sched=sched, layer_size=64)
    assert np.array_equal(e[idx], o.e) and np.array_equal(conv[idx], o.converged)
    assert np.array_equal(it[idx], o.iters)
