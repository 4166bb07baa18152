"""CPU oracle for syndrome-based normalized min-sum (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  It wraps ``oracle.c`` (plain scalar C, a literal
restatement of Algorithm 1, Section 2) and adds pure-Python brute-force
decoders used to pin the oracle itself:

* ``min_weight_decode``: exhaustive minimum-weight solution of H e = s;
* ``max_product_tree``: exact per-bit max-product values W_b(n) = minimum
  weight of an e with H e = s and e_n = b (brute force).

On a tree-shaped Tanner graph, min-sum with alpha = 1 and enough iterations
is exact max-product, so Q_n = gamma * (W_1(n) - W_0(n)) for a uniform prior
gamma -- a classical result on belief propagation on trees (Pearl 1988;
Wiberg 1996) used here as the oracle's exact reference.
"""
from __future__ import annotations

import ctypes as C
import itertools
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        _declare(_lib)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _declare(L):
    vp, i32, f32 = C.c_void_p, C.c_int, C.c_float
    L.orc_flood_f32.argtypes = [i32, i32, vp, i32, vp, vp, f32, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, i32]
    L.orc_flood_i8.argtypes = [i32, i32, vp, i32, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, i32]
    L.orc_layered_f32.argtypes = [i32, i32, vp, i32, vp, vp, f32, i32, vp, i32, i32, vp, vp, vp, vp, i32]
    L.orc_layered_i8.argtypes = [i32, i32, vp, i32, vp, vp, i32, i32, i32, vp, i32, i32, vp, vp, vp, vp, i32]
    L.orc_flood_i16.argtypes = L.orc_flood_i8.argtypes
    L.orc_layered_i16.argtypes = L.orc_layered_i8.argtypes
    L.orc_nms_forward_f64.argtypes = [i32, i32, vp, i32, vp, vp, vp, i32, vp, vp, i32]
    L.orc_nms_adjoint_f64.argtypes = [i32, i32, vp, i32, vp, vp, i32, vp, vp, vp, vp]
    L.orc_syndrome.argtypes = [i32, i32, vp, i32, vp, vp]
    L.orc_edge_count.argtypes = [i32, i32, vp]
    for f in ("orc_flood_f32", "orc_flood_i8", "orc_layered_f32", "orc_layered_i8", "orc_flood_i16",
              "orc_layered_i16",
              "orc_nms_forward_f64", "orc_nms_adjoint_f64", "orc_syndrome", "orc_edge_count"):
        getattr(L, f).restype = C.c_int


def _threads(nthreads):
    return int(nthreads or os.cpu_count() or 1)


def _prep(H, syn):
    H = np.ascontiguousarray(np.asarray(H, dtype=np.uint8))
    syn = np.ascontiguousarray(np.asarray(syn, dtype=np.uint8))
    if syn.ndim == 1:
        syn = syn[None, :]
    return H, syn


def _prior_f32(prior, B, n):
    p = np.asarray(prior, dtype=np.float32)
    if p.ndim == 0:
        p = np.full((B, n), p, dtype=np.float32)
    elif p.ndim == 1:
        p = np.repeat(p[:, None], n, axis=1) if p.size == B and B != n else np.broadcast_to(p, (B, n))
    return np.ascontiguousarray(p, dtype=np.float32)


class Result:
    def __init__(self, e, converged, iters, Q):
        self.e, self.converged, self.iters, self.Q = e, converged, iters, Q


def flood_f32(H, syn, prior, alpha=0.75, max_iters=32, early_stop=True, weights=None,
              want_Q_all=False, want_q_traj=False, nthreads=None):
    """Flooding min-sum, FP32.  prior: scalar, [B] per shot or [B, n].

    weights [T][nnz] (T <= max_iters) replace alpha in iterations 1..T;
    iterations T+1..max_iters use alpha (neural min-sum, then plain min-sum
    continuing from its messages)."""
    H, syn = _prep(H, syn)
    m, n = H.shape
    B = syn.shape[0]
    prior = _prior_f32(prior, B, n)
    nnz = int(lib().orc_edge_count(m, n, _p(H)))
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    if w is not None:
        assert w.ndim == 2 and w.shape[1] == nnz and 1 <= w.shape[0] <= max_iters
    e = np.zeros((B, n), np.uint8)
    conv = np.zeros(B, np.uint8)
    it = np.zeros(B, np.int32)
    Q = np.zeros((B, n), np.float32)
    Qa = np.zeros((max_iters, B, n), np.float32) if want_Q_all else None
    qt = np.zeros((max_iters, B, nnz), np.float32) if want_q_traj else None
    rc = lib().orc_flood_f32(m, n, _p(H), B, _p(syn), _p(prior), float(alpha), _p(w),
                             0 if w is None else int(w.shape[0]),
                             int(max_iters), int(bool(early_stop)), _p(e), _p(conv), _p(it),
                             _p(Q), _p(Qa), _p(qt), _threads(nthreads))
    assert rc == 0
    r = Result(e, conv, it, Q)
    r.Q_all, r.q_traj = Qa, qt
    return r


def alpha_fraction(alpha: float):
    """alpha = num / 2^sh with the smallest sh <= 8, or ValueError."""
    for sh in range(0, 9):
        num = alpha * (1 << sh)
        if num == int(num):
            return int(num), sh
    raise ValueError(f"alpha={alpha} is not a dyadic fraction with denominator <= 256")


def _prior_fx(prior, dtype, n):
    p = np.asarray(prior, dtype=dtype)
    if p.ndim == 1:
        p = np.repeat(p[:, None], n, axis=1)
    return np.ascontiguousarray(p)


def _flood_fx(fn, dtype, H, syn, prior, alpha, max_iters, early_stop, nthreads):
    H, syn = _prep(H, syn)
    m, n = H.shape
    B = syn.shape[0]
    p = _prior_fx(prior, dtype, n)
    num, sh = alpha_fraction(alpha)
    e = np.zeros((B, n), np.uint8)
    conv = np.zeros(B, np.uint8)
    it = np.zeros(B, np.int32)
    Q = np.zeros((B, n), np.float32)
    rc = fn(m, n, _p(H), B, _p(syn), _p(p), num, sh, int(max_iters),
            int(bool(early_stop)), _p(e), _p(conv), _p(it), _p(Q), _threads(nthreads))
    assert rc == 0
    return Result(e, conv, it, Q)


def flood_i8(H, syn, prior_q4, alpha=0.75, max_iters=32, early_stop=True, nthreads=None):
    """Flooding, int8 messages saturated to [-127, 127], Q4 priors; Q reported as Q/16."""
    return _flood_fx(lib().orc_flood_i8, np.int8, H, syn, prior_q4, alpha, max_iters, early_stop, nthreads)


def flood_i16(H, syn, prior_q8, alpha=0.75, max_iters=32, early_stop=True, nthreads=None):
    """Flooding, int16 messages saturated to [-32767, 32767], Q8 priors; Q reported as Q/256."""
    return _flood_fx(lib().orc_flood_i16, np.int16, H, syn, prior_q8, alpha, max_iters, early_stop, nthreads)


def _layers(m, layer_size):
    if m % layer_size:
        raise ValueError("layer size must divide m")
    return np.arange(0, m + 1, layer_size, dtype=np.int32)


def layered_f32(H, syn, prior, layer_size, alpha=0.75, max_iters=32, early_stop=True, nthreads=None):
    H, syn = _prep(H, syn)
    m, n = H.shape
    B = syn.shape[0]
    prior = _prior_f32(prior, B, n)
    lp = _layers(m, layer_size)
    e = np.zeros((B, n), np.uint8)
    conv = np.zeros(B, np.uint8)
    it = np.zeros(B, np.int32)
    Q = np.zeros((B, n), np.float32)
    rc = lib().orc_layered_f32(m, n, _p(H), B, _p(syn), _p(prior), float(alpha), lp.size - 1, _p(lp),
                               int(max_iters), int(bool(early_stop)), _p(e), _p(conv), _p(it), _p(Q),
                               _threads(nthreads))
    assert rc == 0
    return Result(e, conv, it, Q)


def _layered_fx(fn, dtype, H, syn, prior, layer_size, alpha, max_iters, early_stop, nthreads):
    H, syn = _prep(H, syn)
    m, n = H.shape
    B = syn.shape[0]
    p = _prior_fx(prior, dtype, n)
    num, sh = alpha_fraction(alpha)
    lp = _layers(m, layer_size)
    e = np.zeros((B, n), np.uint8)
    conv = np.zeros(B, np.uint8)
    it = np.zeros(B, np.int32)
    Q = np.zeros((B, n), np.float32)
    rc = fn(m, n, _p(H), B, _p(syn), _p(p), num, sh, lp.size - 1, _p(lp),
            int(max_iters), int(bool(early_stop)), _p(e), _p(conv), _p(it), _p(Q), _threads(nthreads))
    assert rc == 0
    return Result(e, conv, it, Q)


def layered_i8(H, syn, prior_q4, layer_size, alpha=0.75, max_iters=32, early_stop=True, nthreads=None):
    return _layered_fx(lib().orc_layered_i8, np.int8, H, syn, prior_q4, layer_size, alpha, max_iters,
                       early_stop, nthreads)


def layered_i16(H, syn, prior_q8, layer_size, alpha=0.75, max_iters=32, early_stop=True, nthreads=None):
    return _layered_fx(lib().orc_layered_i16, np.int16, H, syn, prior_q8, layer_size, alpha, max_iters,
                       early_stop, nthreads)


def nms_forward_f64(H, syn, prior, weights, nthreads=None):
    """Neural min-sum forward in float64: (Q_all [T][B][n], q_traj [T][B][nnz])."""
    H, syn = _prep(H, syn)
    m, n = H.shape
    B = syn.shape[0]
    w = np.ascontiguousarray(weights, dtype=np.float64)
    T, nnz = w.shape
    pr = np.ascontiguousarray(_prior_f32(prior, B, n), dtype=np.float64) if np.asarray(prior).dtype != np.float64 \
        else np.ascontiguousarray(np.broadcast_to(np.asarray(prior, np.float64).reshape(B, -1), (B, n)))
    Qa = np.zeros((T, B, n), np.float64)
    qt = np.zeros((T, B, nnz), np.float64)
    rc = lib().orc_nms_forward_f64(m, n, _p(H), B, _p(syn), _p(pr), _p(w), T, _p(Qa), _p(qt),
                                   _threads(nthreads))
    assert rc == 0
    return Qa, qt


def nms_adjoint_f64(H, syn, weights, q_traj, G):
    """dL/dw [T][nnz] (summed over shots) and the sum of |per-shot terms|."""
    H, syn = _prep(H, syn)
    m, n = H.shape
    B = syn.shape[0]
    w = np.ascontiguousarray(weights, dtype=np.float64)
    T, nnz = w.shape
    qt = np.ascontiguousarray(q_traj, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    assert qt.shape == (T, B, nnz) and G.shape == (T, B, n)
    gw = np.zeros((T, nnz), np.float64)
    ga = np.zeros((T, nnz), np.float64)
    rc = lib().orc_nms_adjoint_f64(m, n, _p(H), B, _p(syn), _p(w), T, _p(qt), _p(G), _p(gw), _p(ga))
    assert rc == 0
    return gw, ga


def syndrome(H, e):
    """Oracle-side s = H e^T mod 2 by a plain double loop."""
    H = np.ascontiguousarray(np.asarray(H, dtype=np.uint8))
    e = np.ascontiguousarray(np.asarray(e, dtype=np.uint8))
    if e.ndim == 1:
        e = e[None, :]
    m, n = H.shape
    s = np.zeros((e.shape[0], m), np.uint8)
    lib().orc_syndrome(m, n, _p(H), e.shape[0], _p(e), _p(s))
    return s


def nms_loss_grad(Q_all, e_true):
    """BCE between e and sigma(-Q) averaged over iterations, shots and bits.

    L = mean_{k,b,n} [ e softplus(Q) + (1-e) softplus(-Q) ];  dL/dQ = (sigma(Q) - (1-e)) / count
    i.e. (e - sigma(-Q)) / count.
    """
    Q = np.asarray(Q_all, dtype=np.float64)
    e = np.asarray(e_true, dtype=np.float64)[None]
    sp = lambda x: np.logaddexp(0.0, x)
    L = np.mean(e * sp(Q) + (1 - e) * sp(-Q))
    G = (e - 1.0 / (1.0 + np.exp(Q))) / Q.size
    return L, G


# ---------------------------------------------------------------------------
# Pure-Python brute force (tiny codes only)
# ---------------------------------------------------------------------------

def all_solutions(H, s):
    """Every e in GF(2)^n with H e = s (n <= 20)."""
    H = np.asarray(H, dtype=np.int64)
    m, n = H.shape
    assert n <= 20
    s = np.asarray(s, dtype=np.int64)
    sols = []
    for bits in itertools.product((0, 1), repeat=n):
        e = np.array(bits, dtype=np.int64)
        if np.array_equal(H.dot(e) % 2, s % 2):
            sols.append(e)
    return np.array(sols, dtype=np.uint8).reshape(-1, n)


def min_weight_decode(H, s):
    sols = all_solutions(H, s)
    if sols.shape[0] == 0:
        return None, None
    w = sols.sum(axis=1)
    return sols[int(np.argmin(w))], int(w.min())


def max_product_tree(H, s):
    """W[b][n] = min weight of e with H e = s and e_n = b (inf if none)."""
    sols = all_solutions(H, s)
    n = np.asarray(H).shape[1]
    W = np.full((2, n), np.inf)
    if sols.shape[0] == 0:
        return W
    w = sols.sum(axis=1)
    for j in range(n):
        for b in (0, 1):
            sel = sols[:, j] == b
            if sel.any():
                W[b, j] = w[sel].min()
    return W
