"""The C-ABI library without a GPU: it loads, exports every function that
include/qldpc.h declares, and its host-only logic behaves as documented
(argument validation happens before any device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "qldpc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qldpc_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    from paper_2508_07879_amd import abi
    names = header_functions()
    assert "qldpc_decode_batch" in names and "qldpc_code_create" in names
    missing = [n for n in names if not hasattr(abi.lib, n)]
    assert not missing, missing


def test_quantize_prior_matches_q4_definition():
    from paper_2508_07879_amd import abi
    from workload import noise
    x = np.array([0.0, -0.0, 0.03125, -0.03125, 3.4761, 4.5951, 100.0, -100.0, 7.96875, -7.9], np.float32)
    x = np.concatenate([x, np.random.default_rng(0).normal(0, 4, 1000).astype(np.float32)])
    assert np.array_equal(abi.qldpc_quantize_prior(x), noise.quantize_q4(x))


def test_default_params():
    from paper_2508_07879_amd import abi
    p = abi.qldpc_default_params()
    assert (p.fmt, p.sched, p.max_iters, p.early_stop, p.prior_mode, p.layout) == (0, 0, 32, 1, 0, 0)
    assert abs(p.alpha - 0.75) < 1e-9
    assert abi.qldpc_version() >= 100


def _create(**kw):
    from paper_2508_07879_amd import abi
    from workload import lp
    c = lp.lp_code(16)
    s = c.hz
    args = dict(m=s.m, n=s.n, row_ptr=s.row_ptr.copy(), col_idx=s.col_idx.copy(), lift_L=16,
                base=s.base.copy())
    args.update(kw)
    return abi.qldpc_code_create(args["m"], args["n"], args["row_ptr"], args["col_idx"],
                                 args["lift_L"], args["base"])


@pytest.mark.parametrize("case", ["cols_unsorted", "col_range", "lift_mismatch", "deg1", "bad_exp"])
def test_code_create_rejects_malformed_input(case):
    from paper_2508_07879_amd import abi
    from workload import lp
    s = lp.lp_code(16).hz
    rp, ci, base = s.row_ptr.copy(), s.col_idx.copy(), s.base.copy()
    kw = {}
    if case == "cols_unsorted":
        ci[0], ci[1] = ci[1], ci[0]
        kw = dict(col_idx=ci)
    elif case == "col_range":
        ci[5] = s.n + 3
        kw = dict(col_idx=ci)
    elif case == "lift_mismatch":
        base[0, np.nonzero(base[0] >= 0)[0][0]] += 1
        kw = dict(base=base % 16 * (base >= 0) - (base < 0))
    elif case == "deg1":
        rp2 = np.concatenate([[0, 1], rp[1:] * 0 + rp[-1]]).astype(np.int32)
        kw = dict(row_ptr=rp2)
    elif case == "bad_exp":
        base[1, np.nonzero(base[1] >= 0)[0][0]] = 16
        kw = dict(base=base)
    with pytest.raises(abi.QldpcError) as ei:
        _create(**kw)
    assert ei.value.status == abi.QLDPC_ERR_INVALID_ARG


def test_code_create_takes_any_valid_matrix_and_refuses_oversized_ones():
    """A valid H without a compiled block pattern, or without lift data at
    all, goes to the edge-list decoder: on a machine without a GPU, creation
    then fails only at the device step.  A code whose messages cannot fit one
    wavefront's LDS even in int8 is refused before any device call."""
    from paper_2508_07879_amd import abi
    from workload import lp
    base = -np.ones((2, 4), np.int64)
    base[0, :3] = [0, 1, 2]
    base[1, 1:] = [3, 0, 1]
    rp, ci = lp.expand_csr(base, 16)
    for lift, b in ((16, base), (0, None)):
        try:
            h = abi.qldpc_code_create(32, 64, rp, ci, lift, b)
            abi.qldpc_code_destroy(h)
        except abi.QldpcError as e:
            assert e.status == abi.QLDPC_ERR_DEVICE, str(e)
    # 40000 checks of degree 2 on a ring: 80000 int8 messages > 64 KB
    m = 40000
    rp = np.arange(0, 2 * m + 1, 2, dtype=np.int32)
    ci = np.stack([np.arange(m), (np.arange(m) + 1) % m], 1)
    ci.sort(axis=1)
    with pytest.raises(abi.QldpcError) as ei:
        abi.qldpc_code_create(m, m, rp, ci.reshape(-1).astype(np.int32), 0, None)
    assert ei.value.status == abi.QLDPC_ERR_UNSUPPORTED


def test_shape_tables_match_the_lp_construction():
    """The kernels' compile-time block pattern equals the workload's LP(A,A*)
    expansion: checked through code_create accepting every L and side up to
    the device allocation (which needs a GPU)."""
    from paper_2508_07879_amd import abi
    from workload import lp
    for L in (16, 32, 64, 128):
        c = lp.lp_code(L)
        for side in (c.hz, c.hx):
            try:
                h = abi.qldpc_code_create(side.m, side.n, side.row_ptr, side.col_idx, L, side.base)
                abi.qldpc_code_destroy(h)
            except abi.QldpcError as e:
                # without a GPU the only acceptable failure is the device step
                assert e.status == abi.QLDPC_ERR_DEVICE, str(e)


def test_quantize_prior_q8_matches_definition():
    from paper_2508_07879_amd import abi
    from workload import noise
    x = np.array([0.0, -0.0, 1 / 512, -1 / 512, 3.4761, 4.5951, 200.0, -200.0, 127.998, -127.9], np.float32)
    x = np.concatenate([x, np.random.default_rng(1).normal(0, 8, 1000).astype(np.float32)])
    q = abi.qldpc_quantize_prior_q8(x)
    assert q.dtype == np.int16 and np.array_equal(q, noise.quantize_q8(x))
    assert q[6] == 32767 and q[7] == -32767


def test_new_entry_points_validate_before_any_device_call():
    from paper_2508_07879_amd import abi
    p = abi.qldpc_default_params()
    with pytest.raises(abi.QldpcError) as ei:
        abi.qldpc_session_create_css(None, None, p, 4)
    assert ei.value.status == abi.QLDPC_ERR_INVALID_ARG
    with pytest.raises(abi.QldpcError) as ei:
        abi.qldpc_nbp_decode_continue(None, 4, 8, None, 32, 0.75, None, None, None, None, None, None, stream=0)
    assert ei.value.status == abi.QLDPC_ERR_INVALID_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
