"""The allocation-free decode entry point (qldpc_decode_batch_static) against
qldpc_decode_batch_ws on the same inputs.  Two calls in a row, the second
with a smaller batch, in the HBM-message layout (asked for explicitly), where
the library's static workspace replaces the caller's (L = 256 in FP32 and
int8, L = 128); the refusal of a batch beyond the static buffer; and the
on-chip layouts AUTO takes (L = 64, and registers at L = 256), which use no
workspace.  Outputs must be bit-identical:
both entry points run the same kernels on the same inputs."""
import numpy as np
import pytest

from workload import bits, lp, noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi  # noqa: E402

_decs = {}


def dec_for(L):
    if L not in _decs:
        _decs[L] = Decoder(lp.lp_code(L).hz)
    return _decs[L]


def inputs(dec, L, shots, p, seed, fmt):
    b = noise.Batch(lp.lp_code(L).hz, seed, np.arange(shots), p)
    syn = torch.from_numpy(np.ascontiguousarray(bits.pack_bits(b.s)).view(np.int32)).cuda()
    pr = torch.from_numpy(b.gamma if fmt == abi.QLDPC_F32 else b.gamma_q4()).cuda()
    return syn, pr


def run(dec, prm, B, syn, pr, static):
    err, conv, it, post = dec.outputs(B, posterior=True)
    if static:
        abi.qldpc_decode_batch_static(dec.handle, prm, B, syn, pr, err, conv, it, post)
    else:
        need = abi.qldpc_decode_workspace_bytes(dec.handle, prm, B)
        ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = ws.data_ptr() + (-ws.data_ptr()) % 256
        abi.qldpc_decode_batch_ws(dec.handle, prm, B, syn, pr, err, conv, it, post, base, need)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (err, conv, it, post)]


def check_pair(L, prm, batches, p, fmt):
    dec = dec_for(L)
    for i, B in enumerate(batches):
        syn, pr = inputs(dec, L, B, p, 700 + 10 * L + i, fmt)
        ref = run(dec, prm, B, syn, pr, static=False)
        got = run(dec, prm, B, syn, pr, static=True)
        for name, x, y in zip(("errors", "converged", "iterations", "posterior"), ref, got):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"L={L} B={B} call {i}: {name} differ"
        assert ref[1].any(), "no shot converged: the comparison would be vacuous"


@pytest.mark.parametrize("fmt,batches", [(abi.QLDPC_F32, (400, 97)), (abi.QLDPC_I8Q4, (1500, 33))])
def test_static_equals_caller_workspace_L256(fmt, batches):
    dec = dec_for(256)
    prm = dec.params(fmt=fmt, layout=abi.QLDPC_LAYOUT_HBM)
    for B in batches:
        assert 0 < abi.qldpc_decode_workspace_bytes(dec.handle, prm, B) <= abi.QLDPC_STATIC_WORKSPACE_BYTES
    check_pair(256, prm, batches, 0.05, fmt)


def test_static_equals_caller_workspace_L128_hbm_layout():
    dec = dec_for(128)
    check_pair(128, dec.params(layout=abi.QLDPC_LAYOUT_HBM), (700, 64), 0.04, abi.QLDPC_F32)


def test_static_refuses_beyond_its_buffer():
    dec = dec_for(256)
    prm = dec.params(layout=abi.QLDPC_LAYOUT_HBM)
    per_shot = 120 * 256 * 4
    B = abi.QLDPC_STATIC_WORKSPACE_BYTES // per_shot + 1
    syn = torch.zeros((B, dec.syn_words), dtype=torch.int32, device="cuda")
    pr = torch.full((B,), 3.0, device="cuda")
    err, conv, it, _ = dec.outputs(B)
    conv.fill_(7)
    with pytest.raises(abi.QldpcError) as ei:
        abi.qldpc_decode_batch_static(dec.handle, prm, B, syn, pr, err, conv, it, None)
    assert ei.value.status == abi.QLDPC_ERR_CAPACITY
    torch.cuda.synchronize()
    assert torch.all(conv == 7)                      # nothing was launched
    abi.qldpc_decode_batch_static(dec.handle, prm, B - 1, syn, pr, err, conv, it, None)
    torch.cuda.synchronize()
    assert torch.all(conv[: B - 1] == 1) and torch.all(conv[B - 1:] == 7)   # zero syndromes converge


def test_static_on_chip_layout_needs_no_workspace():
    dec = dec_for(64)
    prm = dec.params()
    assert abi.qldpc_decode_workspace_bytes(dec.handle, prm, 4096) == 0
    check_pair(64, prm, (4096, 100), 0.03, abi.QLDPC_F32)
    dec256 = dec_for(256)
    assert abi.qldpc_decode_workspace_bytes(dec256.handle, dec256.params(), 4096) == 0
    check_pair(256, dec256.params(), (600, 64), 0.05, abi.QLDPC_F32)
