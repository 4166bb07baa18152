"""Decode calls captured in a hipGraph (through torch.cuda.graph): the C-ABI
decode entry points launch kernels only (no allocation, no memset, no
synchronisation), so a captured decode replays on whatever the static input
buffers hold.  Each layout is captured once and replayed three times on
alternating inputs, with eager decodes between the replays; every replay
must equal the eager decode of the same inputs bit for bit."""
import numpy as np
import pytest

from workload import bits, lp, noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi  # noqa: E402

REG, BLOCK, HBM = abi.QLDPC_LAYOUT_WAVE_REG, abi.QLDPC_LAYOUT_BLOCK, abi.QLDPC_LAYOUT_HBM
_decs = {}


def dec_for(L):
    if L not in _decs:
        _decs[L] = Decoder(lp.lp_code(L).hz)
    return _decs[L]


def inputs(L, B, p, seed, fmt):
    b = noise.Batch(lp.lp_code(L).hz, seed, np.arange(B), p)
    syn = torch.from_numpy(np.ascontiguousarray(bits.pack_bits(b.s)).view(np.int32)).cuda()
    pr = {0: b.gamma, 1: b.gamma_q4(), 2: b.gamma_q8()}[fmt]
    return syn, torch.from_numpy(np.ascontiguousarray(pr)).cuda()


@pytest.mark.parametrize("L,B,fmt,sched,layout,nw", [
    (64, 4096, 0, 0, REG, 0),       # the benchmark's register kernel
    (64, 2048, 1, 1, REG, 0),       # int8 layered, registers
    (64, 100, 0, 0, BLOCK, 16),     # workgroup decoder (small batches)
    (128, 1024, 0, 0, REG, 0),      # two wavefronts per shot
    (256, 256, 2, 0, REG, 0),       # four wavefronts per shot, int16
    (256, 128, 0, 0, HBM, 0),       # messages in a caller workspace
])
def test_captured_decode_replays_equal_eager(L, B, fmt, sched, layout, nw):
    dec = dec_for(L)
    prm = dec.params(fmt=fmt, sched=sched, layout=layout, waves_per_shot=nw)
    need = abi.qldpc_decode_workspace_bytes(dec.handle, prm, B)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda") if need else None
    ws_ptr = (ws.data_ptr() + (-ws.data_ptr()) % 256) if need else None
    ins = [inputs(L, B, 0.05, 500 + L + k, fmt) for k in range(2)]

    def decode(syn, pr, outs):
        if need:
            abi.qldpc_decode_batch_ws(dec.handle, prm, B, syn, pr, *outs, None, ws_ptr, need)
        else:
            abi.qldpc_decode_batch(dec.handle, prm, B, syn, pr, *outs, None)

    refs = []
    for syn, pr in ins:
        outs = dec.outputs(B)[:3]
        decode(syn, pr, outs)
        torch.cuda.synchronize()
        refs.append([x.clone() for x in outs])
        assert outs[1].any(), "no shot converged: the comparison would be vacuous"

    s_syn, s_pr = ins[0][0].clone(), ins[0][1].clone()
    s_out = dec.outputs(B)[:3]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        decode(s_syn, s_pr, s_out)
    for step, k in enumerate((1, 0, 1)):
        s_syn.copy_(ins[k][0])
        s_pr.copy_(ins[k][1])
        for x in s_out:
            x.fill_(0x5A)                       # stale outputs must be overwritten
        g.replay()
        other = dec.outputs(B)[:3]              # eager work between replays
        decode(ins[1 - k][0], ins[1 - k][1], other)
        torch.cuda.synchronize()
        for name, x, y in zip(("errors", "converged", "iterations"), s_out, refs[k]):
            assert torch.equal(x, y), f"L={L} layout={layout} replay {step}: {name} differ from the eager decode"
        for x, y in zip(other, refs[1 - k]):
            assert torch.equal(x, y)
