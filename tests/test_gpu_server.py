"""Continuous-batching server: every request's result equals decoding it
alone (plain min-sum through qldpc_decode_batch, neural min-sum through
qldpc_nbp_decode) whatever else shares its micro-batch; admission refuses
work beyond the queue and the HBM budget; a micro-batch whose launch fails
(failure injected on the host, before anything is enqueued) completes every
affected request with an error status and leaves its buffers untouched; the
Poisson load generator runs."""
import time

import numpy as np
import pytest

from workload import bits, lp, noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_07879_amd import Decoder, abi, nms  # noqa: E402

from gpu_util import to_dev  # noqa: E402

LS = (32, 64, 128)
T = 8
_st = {}


def setup():
    if not _st:
        codes = [lp.lp_code(L) for L in LS]
        decs = [Decoder(c.hz) for c in codes]
        rng = np.random.default_rng(5)
        w = [to_dev(rng.uniform(0.6, 0.9, size=(T, c.hz.nnz)).astype(np.float32)) for c in codes]
        _st.update(codes=codes, decs=decs, w=w)
    return _st


def alone(st, c, decoder, syn_words, prior):
    dec = st["decs"][c]
    B = syn_words.shape[0]
    syn = to_dev(syn_words.view(np.int32))
    pr = to_dev(prior)
    err, conv, it, _ = dec.outputs(B)
    prm = dec.params(max_iters=32)
    if decoder == 0:
        abi.qldpc_decode_batch(dec.handle, prm, B, syn, pr, err, conv, it, None)
    else:
        used = torch.empty(B, dtype=torch.uint8, device="cuda")
        abi.qldpc_nbp_decode(dec.handle, B, T, st["w"][c], prm, syn, pr, err, conv, it, used)
    torch.cuda.synchronize()
    return err.cpu().numpy().view(np.uint32), conv.cpu().numpy(), it.cpu().numpy()


def test_requests_equal_alone_results():
    st = setup()
    prm = st["decs"][0].params(max_iters=32)
    srv = abi.qldpc_server_create([d.handle for d in st["decs"]], prm, nms_weights=st["w"], nms_T=T,
                                  max_inflight=3, max_batch_shots=256, queue_capacity=1000)
    try:
        rng = np.random.default_rng(11)
        reqs = []
        for i in range(120):
            c = int(rng.integers(0, 3))
            dec = int(rng.integers(0, 2))
            ns = int(rng.choice([1, 7, 64]))
            code = st["codes"][c]
            b = noise.Batch(code.hz, 1000 + i, np.arange(ns), float(rng.uniform(0.01, 0.08)))
            syn = np.ascontiguousarray(bits.pack_bits(b.s))
            pr = np.ascontiguousarray(b.gamma)
            err = np.zeros((ns, (code.n + 31) // 32), np.uint32)
            conv = np.full(ns, 9, np.uint8)
            it = np.zeros(ns, np.uint8)
            reqs.append((c, dec, syn, pr, err, conv, it))
            abi.qldpc_server_submit(srv, c, dec, ns, syn, pr, err, conv, it, req_id=i)
        got = {}
        t0 = time.time()
        while len(got) < len(reqs) and time.time() - t0 < 60:
            for q in abi.qldpc_server_poll(srv):
                got[q.req_id] = q
                assert q.status == 0 and q.t_done_ns >= q.t_submit_ns
            time.sleep(0.001)
        assert len(got) == len(reqs)
        for i, (c, dec, syn, pr, err, conv, it) in enumerate(reqs):
            e1, c1, i1 = alone(st, c, dec, syn, pr)
            assert np.array_equal(err, e1) and np.array_equal(conv, c1) and np.array_equal(it, i1), i
    finally:
        abi.qldpc_server_destroy(srv)


def test_admission_limits():
    st = setup()
    prm = st["decs"][0].params(max_iters=32)
    with pytest.raises(abi.QldpcError) as ei:
        abi.qldpc_server_create([d.handle for d in st["decs"]], prm, hbm_budget=1000, max_batch_shots=256)
    assert ei.value.status == abi.QLDPC_ERR_CAPACITY
    srv = abi.qldpc_server_create([d.handle for d in st["decs"]], prm, max_inflight=1, max_batch_shots=64,
                                  queue_capacity=4)
    try:
        slots, slot_bytes, _, _ = abi.qldpc_server_info(srv)
        assert slots == 1 and slot_bytes > 0
        code = st["codes"][1]
        b = noise.Batch(code.hz, 7, np.arange(64), 0.08)
        syn = np.ascontiguousarray(bits.pack_bits(b.s))
        pr = np.ascontiguousarray(b.gamma)
        outs = [np.zeros((64, (code.n + 31) // 32), np.uint32) for _ in range(64)]
        refused = 0
        for i in range(64):
            try:
                abi.qldpc_server_submit(srv, 1, 0, 64, syn, pr, outs[i], None, None, req_id=i)
            except abi.QldpcError as e:
                assert e.status == abi.QLDPC_ERR_CAPACITY
                refused += 1
        assert refused > 0
        with pytest.raises(abi.QldpcError) as ei:
            abi.qldpc_server_submit(srv, 1, 1, 1, syn, pr)        # no neural weights configured
        assert ei.value.status == abi.QLDPC_ERR_UNSUPPORTED
        with pytest.raises(abi.QldpcError) as ei:
            abi.qldpc_server_submit(srv, 1, 0, 65, syn, pr)       # larger than a micro-batch
        assert ei.value.status == abi.QLDPC_ERR_INVALID_ARG
        n = 0
        t0 = time.time()
        while n < 64 - refused and time.time() - t0 < 30:
            n += len(abi.qldpc_server_poll(srv))
            time.sleep(0.001)
        assert n == 64 - refused
    finally:
        abi.qldpc_server_destroy(srv)


def test_poisson_loadgen_runs():
    st = setup()
    prm = st["decs"][0].params(max_iters=32)
    srv = abi.qldpc_server_create([d.handle for d in st["decs"]], prm, nms_weights=st["w"], nms_T=T,
                                  max_inflight=4, max_batch_shots=2048, queue_capacity=100000)
    try:
        pools_s, pools_p = [], []
        for c, code in enumerate(st["codes"]):
            b = noise.Batch(code.hz, 77 + c, np.arange(512), 0.04)
            pools_s.append(np.ascontiguousarray(bits.pack_bits(b.s)))
            pools_p.append(np.ascontiguousarray(b.gamma))
        res, lat = abi.qldpc_server_loadgen(srv, 2e5, 0.5, pools_s, pools_p, seed=3, lat_cap=100000)
        assert res["requests"] > 500 and res["rejected"] == 0
        assert 0 < res["p50_us"] <= res["p99_us"] <= res["max_us"]
        assert lat.size == res["requests"] and np.all(lat > 0)
        print(res)
    finally:
        abi.qldpc_server_destroy(srv)


def test_failed_launch_completes_with_error(monkeypatch):
    st = setup()
    prm = st["decs"][0].params(max_iters=32)
    code = st["codes"][1]
    with pytest.raises(abi.QldpcError) as ei:            # no neural kernel for L = 16
        c16 = Decoder(lp.lp_code(16).hz)
        abi.qldpc_server_create([c16.handle], prm, nms_weights=[st["w"][0]], nms_T=T, max_batch_shots=64)
    assert ei.value.status == abi.QLDPC_ERR_UNSUPPORTED
    monkeypatch.setenv("QLDPC_TEST_FAIL_LAUNCH", "2")    # the second micro-batch fails to launch
    srv = abi.qldpc_server_create([d.handle for d in st["decs"]], prm, max_inflight=1, max_batch_shots=64,
                                  queue_capacity=100)
    monkeypatch.delenv("QLDPC_TEST_FAIL_LAUNCH")
    try:
        nreq = 6
        reqs, submitted = [], []
        for i in range(nreq):
            b = noise.Batch(code.hz, 300 + i, np.arange(64), 0.03)
            syn = np.ascontiguousarray(bits.pack_bits(b.s))
            pr = np.ascontiguousarray(b.gamma)
            err = np.full((64, (code.n + 31) // 32), 0xABABABAB, np.uint32)
            conv = np.full(64, 7, np.uint8)
            it = np.full(64, 7, np.uint8)
            reqs.append((syn, pr, err, conv, it))
            try:
                abi.qldpc_server_submit(srv, 1, 0, 64, syn, pr, err, conv, it, req_id=i)
                submitted.append(i)
            except abi.QldpcError as e:              # submitted after the failure
                assert e.status == abi.QLDPC_ERR_DEVICE
        got = {}
        t0 = time.time()
        status = abi.QLDPC_OK
        while len(got) < len(submitted) and time.time() - t0 < 30:
            out, status = abi.qldpc_server_poll(srv, raise_errors=False)
            for q in out:
                got[q.req_id] = q.status
            time.sleep(0.001)
        assert sorted(got) == submitted
        assert status == abi.QLDPC_ERR_DEVICE
        assert got[0] == abi.QLDPC_OK
        e1, c1, i1 = alone(st, 1, 0, reqs[0][0], reqs[0][1])
        assert np.array_equal(reqs[0][2], e1) and np.array_equal(reqs[0][3], c1)
        for i in submitted[1:]:
            assert got[i] == abi.QLDPC_ERR_DEVICE
            assert np.all(reqs[i][2] == 0xABABABAB) and np.all(reqs[i][3] == 7) and np.all(reqs[i][4] == 7)
        with pytest.raises(abi.QldpcError) as ei:
            abi.qldpc_server_submit(srv, 1, 0, 64, reqs[0][0], reqs[0][1], req_id=99)
        assert ei.value.status == abi.QLDPC_ERR_DEVICE
    finally:
        abi.qldpc_server_destroy(srv)
