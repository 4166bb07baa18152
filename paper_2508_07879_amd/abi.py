"""ctypes binding of the C ABI in include/qldpc.h (argument marshalling only).

Each function keeps the C name and argument order.  Device buffers are
passed as torch CUDA tensors (their data pointers); the stream defaults to
torch's current stream.  Every decode step runs in the HIP library; if the
library is missing this module raises on import.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqldpc.so")

QLDPC_OK = 0
QLDPC_ERR_INVALID_ARG = 1
QLDPC_ERR_UNSUPPORTED = 2
QLDPC_ERR_OUT_OF_MEMORY = 3
QLDPC_ERR_DEVICE = 4
QLDPC_ERR_CAPACITY = 5
QLDPC_ERR_NOT_READY = 6

QLDPC_F32, QLDPC_I8Q4, QLDPC_I16Q8 = 0, 1, 2
QLDPC_FLOOD, QLDPC_LAYERED = 0, 1
QLDPC_PRIOR_PER_SHOT, QLDPC_PRIOR_PER_BIT = 0, 1
QLDPC_LAYOUT_AUTO, QLDPC_LAYOUT_WAVE, QLDPC_LAYOUT_BLOCK, QLDPC_LAYOUT_WAVE_REG, QLDPC_LAYOUT_HBM = 0, 1, 2, 3, 4
QLDPC_IO_COPY, QLDPC_IO_MAPPED, QLDPC_IO_RESIDENT = 0, 1, 2


class QldpcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qldpc status {status}: {msg}")
        self.status = status


class qldpc_code_desc(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("col_idx", C.POINTER(C.c_int32)),
                ("lift_L", C.c_int32), ("base_m", C.c_int32), ("base_n", C.c_int32),
                ("base_exp", C.POINTER(C.c_int32))]


class qldpc_decode_params(C.Structure):
    _fields_ = [("fmt", C.c_int32), ("sched", C.c_int32), ("alpha", C.c_float),
                ("max_iters", C.c_int32), ("early_stop", C.c_int32),
                ("prior_mode", C.c_int32), ("layout", C.c_int32), ("waves_per_shot", C.c_int32)]


class qldpc_server_config(C.Structure):
    _fields_ = [("codes", C.POINTER(C.c_void_p)), ("ncodes", C.c_int32),
                ("nms_weights", C.POINTER(C.c_void_p)), ("nms_T", C.c_int32),
                ("params", qldpc_decode_params), ("hbm_budget", C.c_size_t),
                ("max_inflight", C.c_int32), ("max_batch_shots", C.c_int32), ("queue_capacity", C.c_int32)]


class qldpc_completion(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("code_id", C.c_int32), ("decoder", C.c_int32), ("nshots", C.c_int32),
                ("status", C.c_int32), ("t_submit_ns", C.c_int64), ("t_done_ns", C.c_int64)]


class qldpc_loadgen_config(C.Structure):
    _fields_ = [("rate_shots_per_s", C.c_double), ("duration_s", C.c_double), ("seed", C.c_uint64),
                ("p_single", C.c_double), ("p_neural", C.c_double), ("ncodes", C.c_int32),
                ("pool_syn", C.POINTER(C.c_void_p)), ("pool_prior", C.POINTER(C.c_void_p)),
                ("pool_size", C.POINTER(C.c_int32))]


class qldpc_loadgen_result(C.Structure):
    _fields_ = [("requests", C.c_int64), ("shots", C.c_int64), ("rejected", C.c_int64),
                ("wall_s", C.c_double), ("offered_s", C.c_double), ("p50_us", C.c_double),
                ("p99_us", C.c_double), ("p999_us", C.c_double), ("mean_us", C.c_double),
                ("max_us", C.c_double), ("shots_per_s", C.c_double)]


def _load():
    # torch loads its own HIP runtime under the unversioned file name; let it
    # initialise first so that libqldpc.so binds to that same runtime (same
    # soname) instead of bringing a second one into the process.
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2508_07879_amd/build.py` "
                          "(the decoder has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "qldpc_last_error": ([], C.c_char_p),
        "qldpc_version": ([], i32),
        "qldpc_default_params": ([C.POINTER(qldpc_decode_params)], None),
        "qldpc_quantize_prior": ([vp, vp, i64], i32),
        "qldpc_quantize_prior_q8": ([vp, vp, i64], i32),
        "qldpc_code_create": ([C.POINTER(qldpc_code_desc), i32, C.POINTER(vp)], i32),
        "qldpc_code_destroy": ([vp], i32),
        "qldpc_code_info": ([vp, vp, vp, vp, vp, vp], i32),
        "qldpc_decode_batch": ([vp, C.POINTER(qldpc_decode_params), i32, vp, vp, vp, vp, vp, vp, vp], i32),
        "qldpc_decode_workspace_bytes": ([vp, C.POINTER(qldpc_decode_params), i32, C.POINTER(C.c_size_t)], i32),
        "qldpc_decode_batch_ws": ([vp, C.POINTER(qldpc_decode_params), i32, vp, vp, vp, vp, vp, vp, vp, C.c_size_t,
                                   vp], i32),
        "qldpc_decode_batch_static": ([vp, C.POINTER(qldpc_decode_params), i32, vp, vp, vp, vp, vp, vp, vp], i32),
        "qldpc_autotune": ([vp, C.POINTER(qldpc_decode_params), i32, vp, vp, vp, vp, vp, vp,
                            C.POINTER(qldpc_decode_params)], i32),
        "qldpc_tune_save": ([vp, C.c_char_p], i32),
        "qldpc_tune_load": ([vp, C.c_char_p], i32),
        "qldpc_session_create": ([vp, C.POINTER(qldpc_decode_params), i32, i32, C.POINTER(vp)], i32),
        "qldpc_session_create_css": ([vp, vp, C.POINTER(qldpc_decode_params), i32, C.POINTER(vp)], i32),
        "qldpc_session_destroy": ([vp], i32),
        "qldpc_session_decode": ([vp, i32, vp, vp, vp, vp, vp], i32),
        "qldpc_session_latency": ([vp, i32, i32, i32, vp, vp, vp], i32),
        "qldpc_mixed_create": ([C.POINTER(vp), i32, C.POINTER(qldpc_decode_params), i32, i32, C.POINTER(vp)], i32),
        "qldpc_mixed_destroy": ([vp], i32),
        "qldpc_mixed_decode": ([vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "qldpc_mixed_set_grid": ([vp, i32, i32], i32),
        "qldpc_mixed_autotune": ([vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i32)], i32),
        "qldpc_server_create": ([C.POINTER(qldpc_server_config), C.POINTER(vp)], i32),
        "qldpc_server_info": ([vp, vp, vp, vp, vp], i32),
        "qldpc_server_submit": ([vp, i32, i32, i32, vp, vp, vp, vp, vp, C.c_uint64], i32),
        "qldpc_server_poll": ([vp, vp, i32, C.POINTER(i32)], i32),
        "qldpc_server_destroy": ([vp], i32),
        "qldpc_server_loadgen": ([vp, C.POINTER(qldpc_loadgen_config), C.POINTER(qldpc_loadgen_result), vp,
                                  i64], i32),
        "qldpc_nbp_workspace_bytes": ([vp, i32, i32, C.POINTER(C.c_size_t)], i32),
        "qldpc_nbp_forward": ([vp, i32, i32, vp, vp, vp, vp, vp, vp], i32),
        "qldpc_nbp_backward": ([vp, i32, i32, vp, vp, vp, vp, vp, vp], i32),
        "qldpc_nbp_decode": ([vp, i32, i32, vp, C.POINTER(qldpc_decode_params), vp, vp, vp, vp, vp, vp, vp], i32),
        "qldpc_nbp_decode_continue": ([vp, i32, i32, vp, i32, C.c_float, vp, vp, vp, vp, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _check(st: int):
    if st != QLDPC_OK:
        raise QldpcError(st, lib.qldpc_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):   # a raw device address
        return C.c_void_p(t)
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def qldpc_version() -> int:
    return int(lib.qldpc_version())


def qldpc_default_params() -> qldpc_decode_params:
    p = qldpc_decode_params()
    lib.qldpc_default_params(C.byref(p))
    return p


def qldpc_quantize_prior(llr: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(llr, dtype=np.float32)
    out = np.empty(x.shape, np.int8)
    _check(lib.qldpc_quantize_prior(x.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p), x.size))
    return out


def qldpc_quantize_prior_q8(llr: np.ndarray) -> np.ndarray:
    """int16 Q8 priors: clamp(round-half-away(256 * llr), -32767, 32767)."""
    x = np.ascontiguousarray(llr, dtype=np.float32)
    out = np.empty(x.shape, np.int16)
    _check(lib.qldpc_quantize_prior_q8(x.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p), x.size))
    return out


def qldpc_code_create(m: int, n: int, row_ptr, col_idx, lift_L: int = 0, base=None, device: int = 0):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    d = qldpc_code_desc()
    d.m, d.n = int(m), int(n)
    d.row_ptr = rp.ctypes.data_as(C.POINTER(C.c_int32))
    d.col_idx = ci.ctypes.data_as(C.POINTER(C.c_int32))
    d.lift_L = int(lift_L)
    if base is not None:
        be = np.ascontiguousarray(base, dtype=np.int32)
        d.base_m, d.base_n = be.shape
        d.base_exp = be.ctypes.data_as(C.POINTER(C.c_int32))
    else:
        d.base_m = d.base_n = 0
        d.base_exp = None
    h = C.c_void_p()
    _check(lib.qldpc_code_create(C.byref(d), int(device), C.byref(h)))
    return h


def qldpc_code_destroy(h) -> None:
    _check(lib.qldpc_code_destroy(h))


def qldpc_code_info(h):
    v = [C.c_int32() for _ in range(5)]
    _check(lib.qldpc_code_info(h, *[C.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


def qldpc_decode_batch(h, params: qldpc_decode_params, batch: int, syndromes, priors, errors,
                       converged, iters_used=None, posterior=None, stream=None) -> None:
    _check(lib.qldpc_decode_batch(h, C.byref(params), int(batch), _ptr(syndromes), _ptr(priors),
                                  _ptr(errors), _ptr(converged), _ptr(iters_used), _ptr(posterior),
                                  _stream(stream)))


def qldpc_decode_workspace_bytes(h, params: qldpc_decode_params, batch: int) -> int:
    n = C.c_size_t()
    _check(lib.qldpc_decode_workspace_bytes(h, C.byref(params), int(batch), C.byref(n)))
    return int(n.value)


def qldpc_decode_batch_ws(h, params: qldpc_decode_params, batch: int, syndromes, priors, errors, converged,
                          iters_used=None, posterior=None, workspace=None, workspace_bytes: int = 0,
                          stream=None) -> None:
    _check(lib.qldpc_decode_batch_ws(h, C.byref(params), int(batch), _ptr(syndromes), _ptr(priors), _ptr(errors),
                                     _ptr(converged), _ptr(iters_used), _ptr(posterior), _ptr(workspace),
                                     int(workspace_bytes), _stream(stream)))


QLDPC_STATIC_WORKSPACE_BYTES = 64 << 20


def qldpc_decode_batch_static(h, params: qldpc_decode_params, batch: int, syndromes, priors, errors,
                              converged, iters_used=None, posterior=None, stream=None) -> None:
    _check(lib.qldpc_decode_batch_static(h, C.byref(params), int(batch), _ptr(syndromes), _ptr(priors),
                                         _ptr(errors), _ptr(converged), _ptr(iters_used), _ptr(posterior),
                                         _stream(stream)))


def qldpc_autotune(h, params: qldpc_decode_params, batch: int, syndromes, priors, errors, converged,
                   iters_used=None, stream=None) -> qldpc_decode_params:
    best = qldpc_decode_params()
    _check(lib.qldpc_autotune(h, C.byref(params), int(batch), _ptr(syndromes), _ptr(priors), _ptr(errors),
                              _ptr(converged), _ptr(iters_used), _stream(stream), C.byref(best)))
    return best


def qldpc_tune_save(h, path: str) -> None:
    _check(lib.qldpc_tune_save(h, path.encode()))


def qldpc_tune_load(h, path: str) -> None:
    _check(lib.qldpc_tune_load(h, path.encode()))


def _np(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def qldpc_session_create(h, params: qldpc_decode_params, max_batch: int, io_mode: int = QLDPC_IO_COPY):
    s = C.c_void_p()
    _check(lib.qldpc_session_create(h, C.byref(params), int(max_batch), int(io_mode), C.byref(s)))
    return s


def qldpc_session_create_css(hz_handle, hx_handle, params: qldpc_decode_params, max_pairs: int):
    s = C.c_void_p()
    _check(lib.qldpc_session_create_css(hz_handle, hx_handle, C.byref(params), int(max_pairs), C.byref(s)))
    return s


def qldpc_session_destroy(s) -> None:
    _check(lib.qldpc_session_destroy(s))


def qldpc_session_decode(s, batch: int, host_syndromes: np.ndarray, host_priors: np.ndarray,
                         host_errors: np.ndarray, host_converged: np.ndarray = None,
                         host_iters: np.ndarray = None) -> None:
    """Host numpy arrays in and out (C-contiguous)."""
    _check(lib.qldpc_session_decode(s, int(batch), _np(host_syndromes), _np(host_priors), _np(host_errors),
                                    _np(host_converged), _np(host_iters)))


def qldpc_session_latency(s, nreq: int, batch: int, pool: int, host_syndromes: np.ndarray,
                          host_priors: np.ndarray) -> np.ndarray:
    lat = np.zeros(int(nreq), np.float64)
    _check(lib.qldpc_session_latency(s, int(nreq), int(batch), int(pool), _np(host_syndromes),
                                     _np(host_priors), _np(lat)))
    return lat


def qldpc_nbp_workspace_bytes(h, batch: int, T: int) -> int:
    n = C.c_size_t()
    _check(lib.qldpc_nbp_workspace_bytes(h, int(batch), int(T), C.byref(n)))
    return int(n.value)


def qldpc_nbp_forward(h, batch: int, T: int, weights, syndromes, priors, posteriors, workspace,
                      stream=None) -> None:
    _check(lib.qldpc_nbp_forward(h, int(batch), int(T), _ptr(weights), _ptr(syndromes), _ptr(priors),
                                 _ptr(posteriors), _ptr(workspace), _stream(stream)))


def qldpc_nbp_backward(h, batch: int, T: int, weights, syndromes, workspace, grad_posteriors, grad_weights,
                       stream=None) -> None:
    _check(lib.qldpc_nbp_backward(h, int(batch), int(T), _ptr(weights), _ptr(syndromes), _ptr(workspace),
                                  _ptr(grad_posteriors), _ptr(grad_weights), _stream(stream)))


def qldpc_nbp_decode(h, batch: int, T: int, weights, fallback, syndromes, priors, errors, converged,
                     iters_used, used_fallback, stream=None) -> None:
    fb = None if fallback is None else C.byref(fallback)
    _check(lib.qldpc_nbp_decode(h, int(batch), int(T), _ptr(weights), fb, _ptr(syndromes), _ptr(priors),
                                _ptr(errors), _ptr(converged), _ptr(iters_used), _ptr(used_fallback),
                                _stream(stream)))


def qldpc_nbp_decode_continue(h, batch: int, T: int, weights, max_iters: int, alpha: float, syndromes, priors,
                              errors, converged, iters_used, used_fallback, stream=None) -> None:
    _check(lib.qldpc_nbp_decode_continue(h, int(batch), int(T), _ptr(weights), int(max_iters), float(alpha),
                                         _ptr(syndromes), _ptr(priors), _ptr(errors), _ptr(converged),
                                         _ptr(iters_used), _ptr(used_fallback), _stream(stream)))


def qldpc_mixed_create(handles, params: qldpc_decode_params, max_batch: int, use_graph: bool = True):
    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    x = C.c_void_p()
    _check(lib.qldpc_mixed_create(arr, len(handles), C.byref(params), int(max_batch), int(bool(use_graph)),
                                  C.byref(x)))
    return x


def qldpc_mixed_destroy(x) -> None:
    _check(lib.qldpc_mixed_destroy(x))


def qldpc_mixed_decode(x, batch: int, shot_code, syn_off, err_off, syndromes, priors, errors, converged,
                       iters_used=None, stream=None) -> None:
    _check(lib.qldpc_mixed_decode(x, int(batch), _ptr(shot_code), _ptr(syn_off), _ptr(err_off), _ptr(syndromes),
                                  _ptr(priors), _ptr(errors), _ptr(converged), _ptr(iters_used), _stream(stream)))


def qldpc_mixed_set_grid(x, reg_waves: int = 0, block_workgroups: int = 0) -> None:
    _check(lib.qldpc_mixed_set_grid(x, int(reg_waves), int(block_workgroups)))


def qldpc_mixed_autotune(x, batch: int, shot_code, syn_off, err_off, syndromes, priors, errors, converged,
                         iters_used=None, stream=None) -> int:
    w = C.c_int32()
    _check(lib.qldpc_mixed_autotune(x, int(batch), _ptr(shot_code), _ptr(syn_off), _ptr(err_off), _ptr(syndromes),
                                    _ptr(priors), _ptr(errors), _ptr(converged), _ptr(iters_used), _stream(stream),
                                    C.byref(w)))
    return int(w.value)


def qldpc_server_create(handles, params: qldpc_decode_params, nms_weights=None, nms_T: int = 0,
                        hbm_budget: int = 0, max_inflight: int = 4, max_batch_shots: int = 4096,
                        queue_capacity: int = 65536):
    """nms_weights: None or a list (one per code) of device tensors / None."""
    cfg = qldpc_server_config()
    codes = (C.c_void_p * len(handles))(*[h.value for h in handles])
    cfg.codes = C.cast(codes, C.POINTER(C.c_void_p))
    cfg.ncodes = len(handles)
    keep = [codes]
    if nms_weights is not None:
        ws = (C.c_void_p * len(handles))(*[None if w is None else w.data_ptr() for w in nms_weights])
        cfg.nms_weights = C.cast(ws, C.POINTER(C.c_void_p))
        keep.append(ws)
    cfg.nms_T = int(nms_T)
    cfg.params = params
    cfg.hbm_budget = int(hbm_budget)
    cfg.max_inflight = int(max_inflight)
    cfg.max_batch_shots = int(max_batch_shots)
    cfg.queue_capacity = int(queue_capacity)
    srv = C.c_void_p()
    _check(lib.qldpc_server_create(C.byref(cfg), C.byref(srv)))
    return srv


def qldpc_server_info(srv):
    a, b, c_, d = C.c_int32(), C.c_size_t(), C.c_int32(), C.c_int64()
    _check(lib.qldpc_server_info(srv, C.byref(a), C.byref(b), C.byref(c_), C.byref(d)))
    return int(a.value), int(b.value), int(c_.value), int(d.value)


def qldpc_server_submit(srv, code_id: int, decoder: int, nshots: int, host_syn, host_prior, host_err=None,
                        host_conv=None, host_iters=None, req_id: int = 0) -> None:
    _check(lib.qldpc_server_submit(srv, int(code_id), int(decoder), int(nshots), _np(host_syn), _np(host_prior),
                                   _np(host_err), _np(host_conv), _np(host_iters), C.c_uint64(req_id)))


def qldpc_server_poll(srv, max_n: int = 1024, raise_errors: bool = True):
    """Completions, oldest first.  A failed server reports its status after
    handing out the completions it holds: raise_errors=False returns
    (completions, status) instead of raising."""
    buf = (qldpc_completion * max_n)()
    n = C.c_int32()
    st = lib.qldpc_server_poll(srv, buf, int(max_n), C.byref(n))
    out = [buf[i] for i in range(n.value)]
    if not raise_errors:
        return out, st
    if st not in (QLDPC_OK, QLDPC_ERR_NOT_READY):
        _check(st)
    return out


def qldpc_server_destroy(srv) -> None:
    _check(lib.qldpc_server_destroy(srv))


def qldpc_server_loadgen(srv, rate: float, duration: float, pools_syn, pools_prior, seed: int = 1,
                         p_single: float = 0.5, p_neural: float = 0.5, lat_cap: int = 0):
    """pools_*: per code host numpy arrays ([pool, words] uint32, [pool] float32)."""
    n = len(pools_syn)
    cfg = qldpc_loadgen_config()
    cfg.rate_shots_per_s, cfg.duration_s, cfg.seed = float(rate), float(duration), int(seed)
    cfg.p_single, cfg.p_neural, cfg.ncodes = float(p_single), float(p_neural), n
    ps = (C.c_void_p * n)(*[a.ctypes.data for a in pools_syn])
    pp = (C.c_void_p * n)(*[a.ctypes.data for a in pools_prior])
    sz = (C.c_int32 * n)(*[int(a.shape[0]) for a in pools_prior])
    cfg.pool_syn = C.cast(ps, C.POINTER(C.c_void_p))
    cfg.pool_prior = C.cast(pp, C.POINTER(C.c_void_p))
    cfg.pool_size = C.cast(sz, C.POINTER(C.c_int32))
    res = qldpc_loadgen_result()
    lat = np.zeros(max(1, int(lat_cap)), np.float64)
    _check(lib.qldpc_server_loadgen(srv, C.byref(cfg), C.byref(res), _np(lat), int(lat_cap)))
    out = {f: getattr(res, f) for f, _ in qldpc_loadgen_result._fields_}
    return out, lat[:min(int(lat_cap), out["requests"])]
