"""Neural min-sum kernels against the CPU oracle.

* Forward: every iteration's posterior equals the oracle's FP32 flooding
  with the same per-edge weights (within 1e-5 relative; the order of
  operations is the same, so in practice bit-exact), for positive weights and
  for weights of mixed sign (a negative weight flips its edge's message);
  weights all alpha give plain min-sum.
* Backward: the FP32 adjoint kernel matches the oracle's FP64 adjoint,
  evaluated on the oracle's own FP32 forward trajectory, to 1e-4 of the sum
  of absolute per-shot terms of each weight's gradient; two runs give
  identical bits.
* Autograd: NeuralMinSum + BCE loss produce the oracle gradient of the same
  loss.
* Inference: early-stopped neural decode plus plain min-sum fallback equals
  the oracle composition shot by shot.
"""
import numpy as np
import pytest

import oracle
from workload import bits, lp, noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi, nms  # noqa: E402

from gpu_util import to_dev  # noqa: E402

_codes = {}


def code(L):
    if L not in _codes:
        c = lp.lp_code(L)
        _codes[L] = (c, c.hz.dense(), Decoder(c.hz))
    return _codes[L]


def weights(seed, T, nnz, lo, hi, neg_frac=0.0):
    """U(lo, hi) weights with a random fraction of entries negated."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(lo, hi, size=(T, nnz)).astype(np.float32)
    if neg_frac:
        flip = rng.random(w.shape) < neg_frac
        w[flip] = -w[flip]
        assert flip.any()
    return w


def forward(dec, b, w):
    T = w.shape[0]
    syn = to_dev(bits.pack_bits(b.s).view(np.int32))
    pr = to_dev(b.gamma)
    wt = to_dev(w.astype(np.float32))
    ws = torch.empty(abi.qldpc_nbp_workspace_bytes(dec.handle, b.B, T), dtype=torch.uint8, device="cuda")
    post = torch.empty((T, b.B, dec.n), dtype=torch.float32, device="cuda")
    abi.qldpc_nbp_forward(dec.handle, b.B, T, wt, syn, pr, post, ws)
    torch.cuda.synchronize()
    return syn, wt, ws, post


@pytest.mark.parametrize("wlo", [0.4, -0.6])
@pytest.mark.parametrize("L", [32, 64, 128])
def test_forward_matches_oracle(L, wlo):
    c, H, dec = code(L)
    b = noise.Batch(c.hz, 41, np.arange(37), 0.05)
    T = 6
    w = np.random.default_rng(L).uniform(wlo, 1.0, size=(T, c.hz.nnz)).astype(np.float32)
    assert (w < 0).any() == (wlo < 0)
    _, _, _, post = forward(dec, b, w)
    o = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=T, early_stop=False, want_Q_all=True)
    got = post.cpu().numpy()
    tol = 1e-5 * np.maximum(np.abs(o.Q_all), np.abs(b.gamma)[None, :, None])
    assert np.all(np.abs(got - o.Q_all) <= tol)
    # weights all alpha: plain min-sum, no early stop
    wa = np.full((T, c.hz.nnz), 0.75, np.float32)
    _, _, _, post_a = forward(dec, b, wa)
    oa = oracle.flood_f32(H, b.s, b.gamma, max_iters=T, early_stop=False, want_Q_all=True)
    assert np.all(np.abs(post_a.cpu().numpy() - oa.Q_all) <= 1e-5 * np.maximum(np.abs(oa.Q_all), 1.0))


@pytest.mark.parametrize("wlo", [0.4, -0.6])
@pytest.mark.parametrize("L", [32, 64, 128])
def test_backward_matches_oracle_adjoint(L, wlo):
    c, H, dec = code(L)
    b = noise.Batch(c.hz, 42, np.arange(24), 0.05)
    T = 5
    rng = np.random.default_rng(100 + L)
    w = rng.uniform(wlo, 1.0, size=(T, c.hz.nnz)).astype(np.float32)
    G = rng.normal(size=(T, b.B, c.n)).astype(np.float32)
    syn, wt, ws, post = forward(dec, b, w)
    gw = torch.empty_like(wt)
    abi.qldpc_nbp_backward(dec.handle, b.B, T, wt, syn, ws, to_dev(G), gw)
    gw2 = torch.empty_like(wt)
    abi.qldpc_nbp_backward(dec.handle, b.B, T, wt, syn, ws, to_dev(G), gw2)
    torch.cuda.synchronize()
    g = gw.cpu().numpy()
    assert np.array_equal(g, gw2.cpu().numpy()), "backward is not bit-reproducible"
    of = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=T, early_stop=False, want_q_traj=True)
    go, ga = oracle.nms_adjoint_f64(H, b.s, w.astype(np.float64), of.q_traj.astype(np.float64),
                                    G.astype(np.float64))
    err = np.abs(g - go)
    tol = 1e-4 * ga + 1e-6
    assert np.all(err <= tol), f"max excess {float((err - tol).max())}"
    assert np.abs(go).max() > 0


def test_autograd_loss_gradient():
    c, H, dec = code(64)
    b = noise.Batch(c.hz, 43, np.arange(32), 0.05)
    T = 4
    w = nms.init_weights(T, c.hz.nnz)
    w.requires_grad_(True)
    syn = to_dev(bits.pack_bits(b.s).view(np.int32))
    pr = to_dev(b.gamma)
    post = nms.NeuralMinSum.apply(dec, w, syn, pr)
    loss = nms.bce_loss(post, to_dev(b.e.astype(np.float32)))
    loss.backward()
    of = oracle.flood_f32(H, b.s, b.gamma, weights=w.detach().cpu().numpy(), max_iters=T, early_stop=False,
                          want_Q_all=True, want_q_traj=True)
    L_or, G = oracle.nms_loss_grad(of.Q_all, b.e)
    assert abs(float(loss.detach()) - L_or) <= 1e-5 * abs(L_or)
    go, ga = oracle.nms_adjoint_f64(H, b.s, w.detach().cpu().numpy().astype(np.float64),
                                    of.q_traj.astype(np.float64), G)
    g = w.grad.cpu().numpy()
    assert np.all(np.abs(g - go) <= 1e-4 * ga + 1e-9)


@pytest.mark.parametrize("L,p,neg", [(32, 0.06, 0.0), (64, 0.03, 0.0), (64, 0.03, 0.002)])
def test_inference_with_fallback(L, p, neg):
    c, H, dec = code(L)
    b = noise.Batch(c.hz, 44, np.arange(200), p)
    T = 8
    w = weights(7, T, c.hz.nnz, 0.6, 0.9, neg)
    syn = to_dev(bits.pack_bits(b.s).view(np.int32))
    pr = to_dev(b.gamma)
    err, conv, it, _ = dec.outputs(b.B)
    used = torch.empty(b.B, dtype=torch.uint8, device="cuda")
    fb = dec.params(max_iters=32, layout=abi.QLDPC_LAYOUT_WAVE)
    abi.qldpc_nbp_decode(dec.handle, b.B, T, to_dev(w), fb, syn, pr, err, conv, it, used)
    torch.cuda.synchronize()
    e = bits.unpack_bits(err.cpu().numpy().view(np.uint32), c.n)
    r1 = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=T, early_stop=True)
    fall = r1.converged == 0
    assert fall.any() and (~fall).any()
    r2 = oracle.flood_f32(H, b.s[fall], b.gamma[fall], max_iters=32, early_stop=True)
    want_e = r1.e.copy()
    want_e[fall] = r2.e
    want_c = r1.converged.copy()
    want_c[fall] = r2.converged
    want_i = r1.iters.copy()
    want_i[fall] = r2.iters
    assert np.array_equal(used.cpu().numpy(), fall.astype(np.uint8))
    assert np.array_equal(e, want_e) and np.array_equal(conv.cpu().numpy(), want_c)
    assert np.array_equal(it.cpu().numpy().astype(np.int32), want_i)


@pytest.mark.parametrize("L,p,neg", [(32, 0.06, 0.0), (64, 0.04, 0.0), (128, 0.04, 0.0), (64, 0.04, 0.002)])
def test_inference_with_continuing_fallback(L, p, neg):
    """Neural weights in iterations 1..T, plain min-sum continuing from the
    neural messages up to 32 iterations: decisions, flags and iteration counts
    equal the oracle's, and the fallback flag marks iterations beyond T."""
    c, H, dec = code(L)
    b = noise.Batch(c.hz, 45, np.arange(160 if L < 128 else 64), p)
    T = 8
    w = weights(8, T, c.hz.nnz, 0.6, 0.9, neg)
    syn = to_dev(bits.pack_bits(b.s).view(np.int32))
    pr = to_dev(b.gamma)
    err, conv, it, _ = dec.outputs(b.B)
    used = torch.empty(b.B, dtype=torch.uint8, device="cuda")
    abi.qldpc_nbp_decode_continue(dec.handle, b.B, T, to_dev(w), 32, 0.75, syn, pr, err, conv, it, used)
    torch.cuda.synchronize()
    e = bits.unpack_bits(err.cpu().numpy().view(np.uint32), c.n)
    o = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=32, early_stop=True)
    its = it.cpu().numpy().astype(np.int32)
    assert np.array_equal(e, o.e) and np.array_equal(conv.cpu().numpy(), o.converged)
    assert np.array_equal(its, o.iters)
    assert np.array_equal(used.cpu().numpy(), (o.iters > T).astype(np.uint8))
    assert (o.iters > T).any() and (o.iters <= T).any()
    with pytest.raises(abi.QldpcError) as ei:          # max_iters below T
        abi.qldpc_nbp_decode_continue(dec.handle, b.B, T, to_dev(w), T - 1, 0.75, syn, pr, err, conv, it, used)
    assert ei.value.status == abi.QLDPC_ERR_INVALID_ARG


def test_training_shape_T16_B4096():
    """The training configuration itself (L = 64, T = 16, 4096 shots, a 2 GB
    saved trajectory): the forward pass on sampled shots equals the oracle's
    posteriors of all 16 iterations; the batch gradient equals the sum of the
    gradients of its 64-shot chunks (each a forward and backward of its own),
    so the reduction over the large batch drops and doubles nothing; one chunk
    of 8 shots equals the FP64 oracle adjoint."""
    c, H, dec = code(64)
    B, T, CH = 4096, 16, 64
    b = noise.Batch(c.hz, 46, np.arange(B), 0.05)
    w = weights(9, T, c.hz.nnz, 0.5, 1.0, 0.001)
    G = np.random.default_rng(47).normal(size=(T, B, c.n)).astype(np.float32)
    syn, wt, ws, post = forward(dec, b, w)
    gw = torch.empty_like(wt)
    abi.qldpc_nbp_backward(dec.handle, B, T, wt, syn, ws, to_dev(G), gw)
    torch.cuda.synchronize()
    g_all = gw.cpu().numpy().astype(np.float64)
    pick = np.array([0, 1, 777, 2048, 3000, B - 2, B - 1])
    o = oracle.flood_f32(H, b.s[pick], b.gamma[pick], weights=w, max_iters=T, early_stop=False, want_Q_all=True)
    got = post.cpu().numpy()[:, pick, :]
    assert np.all(np.abs(got - o.Q_all) <= 1e-5 * np.maximum(np.abs(o.Q_all), np.abs(b.gamma[pick])[None, :, None]))
    del post, ws
    g_sum = np.zeros_like(g_all)
    g_abs = np.zeros_like(g_all)
    for lo in range(0, B, CH):
        bc = noise.Batch(c.hz, 46, np.arange(lo, lo + CH), 0.05)
        s_c, w_c, ws_c, _ = forward(dec, bc, w)
        gc = torch.empty_like(w_c)
        abi.qldpc_nbp_backward(dec.handle, CH, T, w_c, s_c, ws_c, to_dev(np.ascontiguousarray(G[:, lo:lo + CH])), gc)
        torch.cuda.synchronize()
        gcn = gc.cpu().numpy().astype(np.float64)
        g_sum += gcn
        g_abs += np.abs(gcn)
    assert np.all(np.abs(g_all - g_sum) <= 1e-4 * g_abs + 1e-5), float(np.abs(g_all - g_sum).max())
    # 8 shots against the FP64 oracle adjoint at T = 16
    b8 = noise.Batch(c.hz, 46, np.arange(8), 0.05)
    s8, w8, ws8, _ = forward(dec, b8, w)
    g8 = torch.empty_like(w8)
    G8 = np.ascontiguousarray(G[:, :8])
    abi.qldpc_nbp_backward(dec.handle, 8, T, w8, s8, ws8, to_dev(G8), g8)
    torch.cuda.synchronize()
    of = oracle.flood_f32(H, b8.s, b8.gamma, weights=w, max_iters=T, early_stop=False, want_q_traj=True)
    go, ga = oracle.nms_adjoint_f64(H, b8.s, w.astype(np.float64), of.q_traj.astype(np.float64),
                                    G8.astype(np.float64))
    assert np.all(np.abs(g8.cpu().numpy() - go) <= 1e-4 * ga + 1e-6)
