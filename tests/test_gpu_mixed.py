"""Mixed-code persistent decoding against the CPU oracle and against
single-code decoding of the same shots (bit-identical: a shot's result does
not depend on its batch mates), eager and through the captured hipGraph
(replayed several times with other device work in between).  The persistent
path proper -- every wavefront and workgroup claiming many tiles in turn --
is checked on small grids and at the benchmark's full 262144-shot size."""
import numpy as np
import pytest

import oracle
from workload import lp
from workload.mixed import MixedBatch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi  # noqa: E402

from gpu_util import gpu_decode, to_dev  # noqa: E402

LS = (16, 32, 64, 128)
_state = {}


def setup():
    if not _state:
        codes = [lp.lp_code(L) for L in LS]
        decs = [Decoder(c.hz) for c in codes]
        _state.update(codes=codes, decs=decs, H=[c.hz.dense() for c in codes])
    return _state


def run_mixed(st, mb, use_graph, reps=1, between=None, grid=None):
    prm = st["decs"][0].params(max_iters=32)
    plan = abi.qldpc_mixed_create([d.handle for d in st["decs"]], prm, mb.B, use_graph)
    try:
        if grid is not None:
            abi.qldpc_mixed_set_grid(plan, *grid)
        dev = dict(cid=to_dev(mb.cid.astype(np.int32)), so=to_dev(mb.syn_off), eo=to_dev(mb.err_off),
                   syn=to_dev(mb.syn.view(np.int32)), pr=to_dev(mb.gamma))
        outs = []
        for r in range(reps):
            err = torch.full((mb.err_words,), -1, dtype=torch.int32, device="cuda")
            conv = torch.full((mb.B,), 7, dtype=torch.uint8, device="cuda")
            it = torch.zeros(mb.B, dtype=torch.uint8, device="cuda")
            # same output buffers on every replay so the graph is reused
            if r == 0:
                bufs = (err, conv, it)
            else:
                bufs[0].fill_(-1)
                bufs[1].fill_(7)
                bufs[2].zero_()
            abi.qldpc_mixed_decode(plan, mb.B, dev["cid"], dev["so"], dev["eo"], dev["syn"], dev["pr"], *bufs)
            torch.cuda.synchronize()
            outs.append(tuple(b.cpu().numpy().copy() for b in bufs))
            if between is not None:
                between()
        return outs
    finally:
        abi.qldpc_mixed_destroy(plan)


def check_against_oracle(st, mb, out):
    err, conv, it = out
    split = mb.split_errors(err.view(np.uint32))
    for c in range(len(LS)):
        idx, _ = mb.e[c]
        if idx.size == 0:
            continue
        o = oracle.flood_f32(st["H"][c], mb.s[c], mb.gamma[idx], max_iters=32)
        assert np.array_equal(split[c], o.e), f"L={LS[c]} decisions differ"
        assert np.array_equal(conv[idx], o.converged) and np.array_equal(it[idx].astype(np.int32), o.iters)
    return split


@pytest.mark.parametrize("use_graph", [False, True])
def test_mixed_batch_matches_oracle_and_single_code(use_graph):
    st = setup()
    mb = MixedBatch(st["codes"], 51, 1500)
    assert len(set(mb.cid.tolist())) == 4
    (out,) = run_mixed(st, mb, use_graph)
    split = check_against_oracle(st, mb, out)
    # the same shots through the single-code decoder, wavefront layout
    for c in range(len(LS)):
        idx, _ = mb.e[c]
        g = gpu_decode(st["decs"][c], mb.s[c], mb.gamma[idx], posterior=False, layout=abi.QLDPC_LAYOUT_WAVE)
        assert np.array_equal(g[0], split[c]) and np.array_equal(g[1], out[1][idx])


def test_graph_replays_match_eager():
    st = setup()
    mb = MixedBatch(st["codes"], 52, 700)
    x = torch.randn(1 << 20, device="cuda")

    def between():
        # unrelated eager device work between replays
        (x * 2.0).sum().item()
        torch.cuda.synchronize()

    eager = run_mixed(st, mb, False)[0]
    graphs = run_mixed(st, mb, True, reps=4, between=between)
    for g in graphs:
        for a_, b_ in zip(eager, g):
            assert np.array_equal(a_, b_)


def test_shot_alone_equals_shot_in_mix():
    st = setup()
    mb = MixedBatch(st["codes"], 53, 400)
    (out,) = run_mixed(st, mb, False)
    split = mb.split_errors(out[0].view(np.uint32))
    for c in range(len(LS)):
        idx, _ = mb.e[c]
        for j in list(range(min(3, idx.size))):
            i = idx[j]
            one = MixedBatch.__new__(MixedBatch)
            one.codes, one.B = mb.codes, 1
            one.cid = mb.cid[i:i + 1]
            one.gamma = mb.gamma[i:i + 1]
            ew = (mb.codes[c].hz.n + 31) // 32
            sw = (mb.codes[c].hz.m + 31) // 32
            one.syn_off = np.zeros(1, np.int64)
            one.err_off = np.zeros(1, np.int64)
            one.syn = mb.syn[mb.syn_off[i]:mb.syn_off[i] + sw].copy()
            one.err_words = ew
            (o1,) = run_mixed(st, one, False)
            assert np.array_equal(o1[0].view(np.uint32), out[0].view(np.uint32)[mb.err_off[i]:mb.err_off[i] + ew])
            assert o1[1][0] == out[1][i] and o1[2][0] == out[2][i]


def test_mixed_autotune_and_bad_code_ids():
    st = setup()
    mb = MixedBatch(st["codes"], 54, 2000)
    prm = st["decs"][0].params(max_iters=32)
    plan = abi.qldpc_mixed_create([d.handle for d in st["decs"]], prm, mb.B, False)
    try:
        cid = mb.cid.astype(np.int32).copy()
        cid[:10] = 99                       # out of range: shot left untouched
        dev = [to_dev(cid), to_dev(mb.syn_off), to_dev(mb.err_off), to_dev(mb.syn.view(np.int32)), to_dev(mb.gamma)]
        err = torch.zeros(mb.err_words, dtype=torch.int32, device="cuda")
        conv = torch.full((mb.B,), 7, dtype=torch.uint8, device="cuda")
        it = torch.zeros(mb.B, dtype=torch.uint8, device="cuda")
        w = abi.qldpc_mixed_autotune(plan, mb.B, *dev, err, conv, it)
        assert w > 0
        conv.fill_(7)
        abi.qldpc_mixed_decode(plan, mb.B, *dev, err, conv, it)
        torch.cuda.synchronize()
        c = conv.cpu().numpy()
        assert np.all(c[:10] == 7) and np.all(c[10:] <= 1)
    finally:
        abi.qldpc_mixed_destroy(plan)


def single_code_all(st, mb, out):
    """Every shot of the mixed result equals its single-code decode."""
    split = mb.split_errors(out[0].view(np.uint32))
    for c in range(len(LS)):
        idx, _ = mb.e[c]
        if idx.size == 0:
            continue
        g = gpu_decode(st["decs"][c], mb.s[c], mb.gamma[idx], posterior=False)
        assert np.array_equal(g[0], split[c]), f"L={LS[c]}: decisions differ from the single-code decode"
        assert np.array_equal(g[1], out[1][idx]) and np.array_equal(g[2], out[2][idx].astype(np.int32))
    return split


def oracle_sample(st, mb, out, split, per_code=24):
    """The first and last shots of each code by index and its unconverged
    shots, up to per_code of each, against the oracle."""
    for c in range(len(LS)):
        idx, _ = mb.e[c]
        if idx.size == 0:
            continue
        k = idx.size
        unconv = np.nonzero(out[1][idx] == 0)[0][:per_code]
        pick = np.unique(np.concatenate([np.arange(min(per_code, k)), np.arange(max(0, k - per_code), k), unconv]))
        o = oracle.flood_f32(st["H"][c], mb.s[c][pick], mb.gamma[idx[pick]], max_iters=32)
        assert np.array_equal(split[c][pick], o.e), f"L={LS[c]}: sampled decisions differ from the oracle"
        assert np.array_equal(out[1][idx[pick]], o.converged)
        assert np.array_equal(out[2][idx[pick]].astype(np.int32), o.iters)


@pytest.mark.parametrize("use_graph", [False, True])
def test_persistent_grids_claim_many_tiles(use_graph):
    """37 register wavefronts per lift and 11 two-wave workgroups for L = 128 over
    6000 shots: every wavefront and workgroup decodes many tiles in turn."""
    st = setup()
    mb = MixedBatch(st["codes"], 55, 6000)
    reg_waves, block_wgs = 37, 11
    for c, L in enumerate(LS):
        n = int((mb.cid == c).sum())
        tiles = -(-n // (64 // L)) if L <= 64 else n
        assert tiles >= 4 * (reg_waves if L <= 64 else block_wgs), (L, n)
    (out,) = run_mixed(st, mb, use_graph, grid=(reg_waves, block_wgs))
    split = single_code_all(st, mb, out)
    oracle_sample(st, mb, out, split)


def test_full_size_mixed_batch():
    """The benchmark's 262144-shot mixed batch at the default grid sizes
    (3072 register wavefronts per lift, 1536 two-wave workgroups for L = 128, so tiles
    outnumber waves for every lift): every shot against its single-code
    decode, a sample against the oracle."""
    st = setup()
    mb = MixedBatch(st["codes"], 20250807 + 99, 262144)
    for c, L in enumerate(LS):
        n = int((mb.cid == c).sum())
        tiles = -(-n // (64 // L)) if L <= 64 else n
        assert tiles > (3072 if L <= 64 else 1536), (L, n)
    (out,) = run_mixed(st, mb, True)
    split = single_code_all(st, mb, out)
    oracle_sample(st, mb, out, split, per_code=16)
