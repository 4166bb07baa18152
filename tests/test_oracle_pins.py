"""Pins for the CPU oracle, each against something other than the oracle.

* Equation (PCM) of Section 2: adjacency sets and degrees as printed.
* Tree-shaped Tanner graphs: with alpha = 1 and enough iterations min-sum is
  exact max-product, so Q_n = gamma (W_1(n) - W_0(n)) with W_b from brute
  force (flooding and layered, FP32, int8 and int16).
* Closed form of the first iteration under a uniform prior (Algorithm 1
  check rule, then the a-posteriori sum), FP32, int8 and int16, including
  per-edge neural weights indexed by row-major edge position.
* Saturation closed form of the fixed-point formats: with s = 0 and a large
  prior every message saturates at its bound, so from the second iteration on
  Q_n = gamma_q + d_v(n) ((3 qmax) >> 2), exactly.
* Exact scale invariance gamma -> 2 gamma (FP32).
* Stopping rule: the reported iteration is the first k with H e^(k) = s,
  converged outputs reproduce the syndrome (checked by an independent
  GF(2) product), inconsistent syndromes never converge.
* Brute-force minimum-weight decoding on tiny loopy codes.
* int8 and int16 flooding against an independent numpy decoder in the
  (min1, min2, Q - r) form, which is exact in integers.
* Neural min-sum: weights all equal to alpha reproduce alpha-MS bit for bit;
  the float64 adjoint matches central finite differences.
"""
import os

import numpy as np
import pytest

import oracle
from workload import lp, noise

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def pcm():
    rows = []
    sv, sc = {}, {}
    for line in open(os.path.join(GOLD, "pcm_eq1.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("Sv"):
            k, v = line[2:].split(":")
            sv[int(k)] = [int(x) for x in v.split()]
        elif line.startswith("Sc"):
            k, v = line[2:].split(":")
            sc[int(k)] = [int(x) for x in v.split()]
        else:
            rows.append([int(x) for x in line.split()])
    return np.array(rows, np.uint8), sv, sc


def random_tree(rng, n_target):
    """Tanner forest with every check of degree >= 2 (n <= n_target)."""
    n = 1
    checks = []
    while n < n_target:
        anchor = int(rng.integers(0, n))
        k = int(min(rng.integers(1, 4), n_target - n))
        new = list(range(n, n + k))
        checks.append([anchor] + new)
        n += k
    H = np.zeros((len(checks), n), np.uint8)
    for i, c in enumerate(checks):
        H[i, c] = 1
    # shuffle rows and columns so that order carries no structure
    H = H[rng.permutation(H.shape[0])][:, rng.permutation(n)]
    return H


def test_pcm_example_adjacency():
    H, sv, sc = pcm()
    assert H.shape == (3, 6)
    assert set(H.sum(1)) == {4} and set(H.sum(0)) == {2}
    for m, cols in sv.items():
        assert np.nonzero(H[m])[0].tolist() == cols
    for n, rows in sc.items():
        assert np.nonzero(H[:, n])[0].tolist() == rows
    assert oracle.lib().orc_edge_count(3, 6, H.ctypes.data_as(oracle.C.c_void_p)) == 12


def test_pcm_example_decodes_every_syndrome_consistently():
    H, _, _ = pcm()
    for s_int in range(8):
        s = np.array([(s_int >> i) & 1 for i in range(3)], np.uint8)
        r = oracle.flood_f32(H, s[None], 2.0, alpha=0.75, max_iters=32)
        e_min, w_min = oracle.min_weight_decode(H, s)
        if e_min is None:
            assert r.converged[0] == 0
            continue
        if r.converged[0]:
            assert np.array_equal(oracle.syndrome(H, r.e)[0], s)
            assert r.e[0].sum() >= w_min


@pytest.mark.parametrize("seed", range(12))
def test_tree_exact_max_product_flood_and_layered(seed):
    rng = np.random.default_rng(100 + seed)
    H = random_tree(rng, int(rng.integers(6, 15)))
    m, n = H.shape
    s = rng.integers(0, 2, size=m).astype(np.uint8)
    W = oracle.max_product_tree(H, s)
    assert np.isfinite(W).all()
    gam = 1.5
    want = gam * (W[1] - W[0])
    iters = 2 * (m + n)
    r = oracle.flood_f32(H, s[None], gam, alpha=1.0, max_iters=iters, early_stop=False)
    assert np.array_equal(r.Q[0], want.astype(np.float32))
    # every row is its own layer; the serial schedule reaches the same fixed point
    rl = oracle.layered_f32(H, s[None], gam, 1, alpha=1.0, max_iters=iters, early_stop=False)
    assert np.array_equal(rl.Q[0], want.astype(np.float32))
    # int8 with a small Q4 prior stays clear of saturation: Q = gq (W1 - W0) / 16
    gq = 4
    r8 = oracle.flood_i8(H, s[None], np.full(n, gq, np.int8)[None], alpha=1.0, max_iters=iters,
                         early_stop=False)
    assert np.array_equal(r8.Q[0] * 16, (gq * (W[1] - W[0])).astype(np.float32))
    rl8 = oracle.layered_i8(H, s[None], np.full(n, gq, np.int8)[None], 1, alpha=1.0, max_iters=iters,
                            early_stop=False)
    assert np.array_equal(rl8.Q[0] * 16, (gq * (W[1] - W[0])).astype(np.float32))
    # int16 with a Q8 prior beyond the int8 range: Q = gq (W1 - W0) / 256
    gq16 = 700
    p16 = np.full(n, gq16, np.int16)[None]
    r16 = oracle.flood_i16(H, s[None], p16, alpha=1.0, max_iters=iters, early_stop=False)
    assert np.array_equal(r16.Q[0] * 256, (gq16 * (W[1] - W[0])).astype(np.float32))
    rl16 = oracle.layered_i16(H, s[None], p16, 1, alpha=1.0, max_iters=iters, early_stop=False)
    assert np.array_equal(rl16.Q[0] * 256, (gq16 * (W[1] - W[0])).astype(np.float32))
    # the hard decision of exact max-product is a minimum-weight solution when unique
    e_min, w_min = oracle.min_weight_decode(H, s)
    if np.all(want != 0):
        assert np.array_equal(r.e[0], e_min)


def test_first_iteration_closed_form_fp32_and_weights():
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 5, np.arange(6), 0.05)
    gam = float(b.gamma[0])
    r = oracle.flood_f32(H, b.s, np.float32(gam), alpha=0.75, max_iters=1, early_stop=False)
    g32 = np.float32(gam)
    a = np.float32(0.75) * g32
    for sh in range(6):
        want = np.empty(c.n, np.float32)
        for nn in range(c.n):
            acc = g32
            for mm in np.nonzero(H[:, nn])[0]:
                acc = np.float32(acc + (-a if b.s[sh, mm] else a))
            want[nn] = acc
        assert np.array_equal(r.Q[sh], want)
    # per-edge weights of both signs: edge index = row-major position of (m, n)
    rng = np.random.default_rng(3)
    w = rng.uniform(-1.0, 1.0, size=(1, c.hz.nnz)).astype(np.float32)
    rw = oracle.flood_f32(H, b.s[:2], np.float32(gam), weights=w, max_iters=1, early_stop=False)
    eidx = -np.ones(H.shape, np.int64)
    eidx[np.nonzero(H)] = np.arange(c.hz.nnz)
    for sh in range(2):
        for nn in range(0, c.n, 7):
            acc = g32
            for mm in np.nonzero(H[:, nn])[0]:
                v = np.float32(w[0, eidx[mm, nn]] * g32)
                acc = np.float32(acc + (-v if b.s[sh, mm] else v))
            assert rw.Q[sh, nn] == acc


def test_first_iteration_closed_form_int8():
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 6, np.arange(4), 0.03)
    gq = int(b.gamma_q4()[0])
    r = oracle.flood_i8(H, b.s, np.full(4, gq, np.int8), max_iters=1, early_stop=False)
    mag = (3 * gq) >> 2
    for sh in range(4):
        want = gq + np.array([sum(-mag if b.s[sh, mm] else mag for mm in np.nonzero(H[:, nn])[0])
                              for nn in range(c.n)])
        assert np.array_equal(r.Q[sh] * 16, want.astype(np.float32))


def test_first_iteration_closed_form_int16():
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 6, np.arange(4), 0.03)
    gq = int(b.gamma_q8()[0])
    assert gq == 890          # round(256 * log(0.97 / 0.03)) = round(889.9)
    r = oracle.flood_i16(H, b.s, np.full(4, gq, np.int16), max_iters=1, early_stop=False)
    mag = (3 * gq) >> 2
    for sh in range(4):
        want = gq + np.array([sum(-mag if b.s[sh, mm] else mag for mm in np.nonzero(H[:, nn])[0])
                              for nn in range(c.n)])
        assert np.array_equal(r.Q[sh] * 256, want.astype(np.float32))


@pytest.mark.parametrize("fmt", ["i8", "i16"])
def test_fixed_point_saturation_closed_form(fmt):
    # s = 0, uniform prior g near the bound: after iteration 1 every excluded
    # sum g + (d-1) r exceeds qmax (d >= 2), so every q is qmax, every r is
    # (3 qmax) >> 2 and Q_n = g + d_v(n) ((3 qmax) >> 2) from then on.
    c = lp.lp_code(16)
    H = c.hz.dense()
    s = np.zeros((2, c.hz.m), np.uint8)
    qmax, g, dt, run, scale = {
        "i8": (127, 120, np.int8, oracle.flood_i8, 16),
        "i16": (32767, 30000, np.int16, oracle.flood_i16, 256)}[fmt]
    dv = H.sum(0).astype(np.int64)
    for k in (2, 3):
        r = run(H, s, np.full(2, g, dt), max_iters=k, early_stop=False)
        want = (g + dv * ((3 * qmax) >> 2)).astype(np.float32)
        assert np.array_equal(r.Q[0] * scale, want) and np.array_equal(r.Q[1] * scale, want)


def test_scale_invariance_fp32():
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 8, np.arange(40), 0.05)
    r1 = oracle.flood_f32(H, b.s, b.gamma)
    r2 = oracle.flood_f32(H, b.s, b.gamma * np.float32(2))
    assert np.array_equal(r1.e, r2.e) and np.array_equal(r1.iters, r2.iters)
    assert np.array_equal(r1.converged, r2.converged)
    assert np.array_equal(r1.Q * 2, r2.Q)
    # and a uniform prior gives the hard decisions of the paper's gamma = 1
    # when the ratio is a power of two
    r4 = oracle.flood_f32(H, b.s, np.float32(4.0))
    r1b = oracle.flood_f32(H, b.s, np.float32(1.0))
    assert np.array_equal(r4.e, r1b.e) and np.array_equal(r4.iters, r1b.iters)


@pytest.mark.parametrize("fmt", ["f32", "i8", "i16", "lf32", "li8", "li16"])
def test_stopping_rule_and_convergence(fmt):
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 9, np.arange(120), 0.04)
    run = {
        "f32": lambda **k: oracle.flood_f32(H, b.s, b.gamma, **k),
        "i8": lambda **k: oracle.flood_i8(H, b.s, b.gamma_q4(), **k),
        "lf32": lambda **k: oracle.layered_f32(H, b.s, b.gamma, 16, **k),
        "li8": lambda **k: oracle.layered_i8(H, b.s, b.gamma_q4(), 16, **k),
        "i16": lambda **k: oracle.flood_i16(H, b.s, b.gamma_q8(), **k),
        "li16": lambda **k: oracle.layered_i16(H, b.s, b.gamma_q8(), 16, **k),
    }[fmt]
    r = run(max_iters=32)
    ok = r.converged == 1
    assert ok.mean() > 0.5
    # converged outputs reproduce the syndrome (independent GF(2) product)
    assert np.array_equal(noise.syndromes(c.hz, r.e[ok]), b.s[ok])
    # non-converged shots report I_max; unconverged outputs do not satisfy s
    assert np.all(r.iters[~ok] == 32)
    assert not np.any(np.all(noise.syndromes(c.hz, r.e[~ok]) == b.s[~ok], axis=1))
    # the reported iteration is the first one whose decision satisfies s
    for k in range(1, 6):
        rk = run(max_iters=k, early_stop=False)
        sat = np.all(noise.syndromes(c.hz, rk.e) == b.s, axis=1)
        stopped_by_k = r.iters <= k
        assert np.array_equal(sat & ~(r.iters < k), (r.iters == k) & ok)
        assert np.all(stopped_by_k[r.iters < k] == True)  # noqa: E712
    # I_max = 1 stops after one iteration
    r1 = run(max_iters=1)
    assert np.all(r1.iters == 1)


def test_inconsistent_syndromes_never_converge():
    c = lp.lp_code(16)
    H = c.hz.dense()
    s = noise.random_syndromes(4, np.arange(64), c.hz.m)
    # consistent iff s in the column space of H; check with the oracle-free rank test
    from workload import gf2
    rk = gf2.rank(H)
    cons = np.array([gf2.rank(np.hstack([H, s[i][:, None]])) == rk for i in range(64)])
    r = oracle.flood_f32(H, s, np.float32(3.0), max_iters=8)
    assert not np.any(r.converged[~cons])


def test_zero_syndrome_returns_zero_at_first_iteration():
    c = lp.lp_code(16)
    H = c.hz.dense()
    s = np.zeros((3, c.hz.m), np.uint8)
    for r in (oracle.flood_f32(H, s, np.float32(2.0)), oracle.flood_i8(H, s, np.full(3, 40, np.int8)),
              oracle.flood_i16(H, s, np.full(3, 640, np.int16)),
              oracle.layered_i16(H, s, np.full(3, 640, np.int16), 16),
              oracle.layered_f32(H, s, np.float32(2.0), 16)):
        assert np.all(r.iters == 1) and np.all(r.converged == 1) and not r.e.any()


@pytest.mark.parametrize("seed", range(6))
def test_tiny_loopy_codes_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    m, n = 5, 12
    while True:
        H = (rng.random((m, n)) < 0.35).astype(np.uint8)
        if H.sum(1).min() >= 2 and H.sum(0).min() >= 1:
            break
    e = (rng.random((40, n)) < 0.1).astype(np.uint8)
    s = ((e.astype(int) @ H.T.astype(int)) % 2).astype(np.uint8)
    r = oracle.flood_f32(H, s, np.float32(2.0))
    for i in range(40):
        _, wmin = oracle.min_weight_decode(H, s[i])
        if r.converged[i]:
            assert np.array_equal(((r.e[i].astype(int) @ H.T) % 2), s[i])
            assert r.e[i].sum() >= wmin


def _numpy_fx_flood(H, s, gq, max_iters, qmax, anum=3, ash=2):
    """Independent fixed-point flooding in the (min1, min2, Q - r) form."""
    m, n = H.shape
    rows = [np.nonzero(H[i])[0] for i in range(m)]
    B = s.shape[0]
    out_e = np.zeros((B, n), np.uint8)
    out_it = np.zeros(B, np.int32)
    for b in range(B):
        r = [np.zeros(len(c), np.int64) for c in rows]
        Q = np.full(n, int(gq[b]), np.int64)
        for k in range(1, max_iters + 1):
            newr = []
            for i, c in enumerate(rows):
                q = np.clip(Q[c] - r[i], -qmax, qmax)
                a = np.abs(q)
                o = np.argsort(a, kind="stable")
                m1, m2 = a[o[0]], a[o[1]]
                neg = (q < 0).astype(np.int64)
                par = (neg.sum() + s[b, i]) & 1
                mag = np.where(np.arange(len(c)) == o[0], m2, m1)
                sgn = 1 - 2 * (par ^ neg)
                newr.append(sgn * ((anum * mag) >> ash))
            Q = np.full(n, int(gq[b]), np.int64)
            for i, c in enumerate(rows):
                np.add.at(Q, c, newr[i])
            r = newr
            e = (Q < 0).astype(np.uint8)
            if np.array_equal((e.astype(int) @ H.T) % 2, s[b]):
                break
        out_e[b], out_it[b] = e, k
    return out_e, out_it


@pytest.mark.parametrize("fmt", ["i8", "i16"])
def test_fixed_point_against_independent_q_minus_r_form(fmt):
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 12, np.arange(24), 0.05)
    if fmt == "i8":
        gq, qmax, r = b.gamma_q4(), 127, oracle.flood_i8(H, b.s, b.gamma_q4(), max_iters=12)
    else:
        gq, qmax, r = b.gamma_q8(), 32767, oracle.flood_i16(H, b.s, b.gamma_q8(), max_iters=12)
    e, it = _numpy_fx_flood(H, b.s, gq, 12, qmax)
    assert np.array_equal(r.e, e) and np.array_equal(r.iters, it)


def test_neural_with_alpha_weights_is_alpha_ms():
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 13, np.arange(30), 0.05)
    T = 6
    w = np.full((T, c.hz.nnz), 0.75, np.float32)
    ra = oracle.flood_f32(H, b.s, b.gamma, max_iters=T, early_stop=False, want_Q_all=True)
    rw = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=T, early_stop=False, want_Q_all=True)
    assert np.array_equal(ra.Q_all, rw.Q_all)
    Qd, _ = oracle.nms_forward_f64(H, b.s, b.gamma.astype(np.float64), w.astype(np.float64))
    assert np.allclose(Qd, ra.Q_all, rtol=1e-5, atol=1e-5 * np.abs(b.gamma).max())


def test_neural_then_plain_continuation():
    """Weights for the first T of I_max iterations: with w = alpha it is plain
    min-sum bit for bit; the first T iterations are the neural decoder's, and
    the iterations after T apply alpha (checked against the double-precision
    neural forward, whose weights are alpha beyond T)."""
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 14, np.arange(30), 0.06)
    T, I = 3, 9
    wa = np.full((T, c.hz.nnz), 0.75, np.float32)
    ra = oracle.flood_f32(H, b.s, b.gamma, max_iters=I, early_stop=False, want_Q_all=True)
    rw = oracle.flood_f32(H, b.s, b.gamma, weights=wa, max_iters=I, early_stop=False, want_Q_all=True)
    assert np.array_equal(ra.Q_all, rw.Q_all)
    rng = np.random.default_rng(5)
    w = rng.uniform(0.4, 1.0, size=(T, c.hz.nnz)).astype(np.float32)
    rn = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=T, early_stop=False, want_Q_all=True)
    rc = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=I, early_stop=False, want_Q_all=True)
    assert np.array_equal(rc.Q_all[:T], rn.Q_all)
    wfull = np.concatenate([w, np.full((I - T, c.hz.nnz), 0.75, np.float32)]).astype(np.float64)
    Qd, _ = oracle.nms_forward_f64(H, b.s, b.gamma.astype(np.float64), wfull)
    assert np.allclose(Qd, rc.Q_all, rtol=1e-5, atol=1e-5 * np.abs(b.gamma).max())
    # with early stop, the reported iteration is the first whose decision satisfies s
    re = oracle.flood_f32(H, b.s, b.gamma, weights=w, max_iters=I, early_stop=True)
    ok = re.converged == 1
    assert np.array_equal(noise.syndromes(c.hz, re.e[ok]), b.s[ok])
    for i in np.nonzero(ok)[0][:10]:
        k = int(re.iters[i])
        assert np.array_equal(rc.Q_all[k - 1, i] < 0, re.e[i].astype(bool))


@pytest.mark.parametrize("wlo", [0.5, -1.0])
def test_neural_adjoint_matches_finite_differences(wlo):
    """Positive weights, and weights of mixed sign (a negative weight flips
    its edge's message; the map stays linear in each weight)."""
    rng = np.random.default_rng(21)
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 14, np.arange(3), 0.06)
    T = 4
    nnz = c.hz.nnz
    w = rng.uniform(wlo, 1.0, size=(T, nnz))
    prior = b.gamma.astype(np.float64)
    G = rng.normal(size=(T, b.B, c.n))
    Qa, qt = oracle.nms_forward_f64(H, b.s, prior, w)
    gw, ga = oracle.nms_adjoint_f64(H, b.s, w, qt, G)
    loss = lambda ww: float(np.sum(G * oracle.nms_forward_f64(H, b.s, prior, ww)[0]))
    idx = [(k, int(e)) for k in range(T) for e in rng.choice(nnz, size=12, replace=False)]
    checked = 0
    for k, e in idx:
        h = 1e-6 * abs(w[k, e])
        wp, wm = w.copy(), w.copy()
        wp[k, e] += h
        wm[k, e] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        # skip points where a comparison flips inside +-h (one-sided slopes disagree)
        f0 = loss(w)
        left, right = (f0 - loss(wm)) / h, (loss(wp) - f0) / h
        if abs(left - right) > 1e-3 * (abs(left) + abs(right) + 1e-9):
            continue
        assert abs(fd - gw[k, e]) <= 1e-6 * max(1.0, abs(gw[k, e]), ga[k, e]), (k, e, fd, gw[k, e])
        checked += 1
    assert checked >= len(idx) * 3 // 4
    # a zero-gradient loss gives a zero gradient
    z, _ = oracle.nms_adjoint_f64(H, b.s, w, qt, np.zeros_like(G))
    assert not z.any()


def test_neural_adjoint_last_iteration_closed_form():
    """dL/dw at iteration T for L = sum_n G_n Q^(T)_n is G_n * sgn * mag."""
    rng = np.random.default_rng(5)
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 15, np.arange(2), 0.05)
    T = 3
    w = rng.uniform(0.5, 1.0, size=(T, c.hz.nnz))
    G = np.zeros((T, 2, c.n))
    G[T - 1] = rng.normal(size=(2, c.n))
    Qa, qt = oracle.nms_forward_f64(H, b.s, b.gamma.astype(np.float64), w)
    gw, _ = oracle.nms_adjoint_f64(H, b.s, w, qt, G)
    rows, cols = np.nonzero(H)
    want = np.zeros(c.hz.nnz)
    for sh in range(2):
        q = qt[T - 1, sh]
        for ei, (mm, nn) in enumerate(zip(rows, cols)):
            others = [f for f in np.nonzero(rows == mm)[0] if f != ei]
            mag = min(abs(q[f]) for f in others)
            sgn = (-1) ** int(b.s[sh, mm]) * np.prod([1 if q[f] >= 0 else -1 for f in others])
            want[ei] += G[T - 1, sh, nn] * sgn * mag
    assert np.allclose(gw[T - 1], want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("fmt", ["i8", "i16"])
def test_layered_saturation_closed_form(fmt):
    """Layered fixed-point schedule with s = 0 and a uniform prior g near the
    bound, block rows as layers.  In the first sweep every check output is
    (3 min) >> 2 with min in {g, qmax}, so every r >= (3 g) >> 2.  From the
    second sweep on, every check input Q - r_old = g + (sum of the other
    d_v - 1 messages) > qmax, so it saturates to qmax, every output is
    (3 qmax) >> 2, and with the posterior kept exactly Q_n = g + d_v(n)
    ((3 qmax) >> 2).  Building Q from the saturated input instead (Q = q + r)
    would give qmax + ((3 qmax) >> 2) for every bit."""
    c = lp.lp_code(16)
    H = c.hz.dense()
    s = np.zeros((2, c.hz.m), np.uint8)
    qmax, g, dt, run, scale = {
        "i8": (127, 120, np.int8, oracle.layered_i8, 16),
        "i16": (32767, 30000, np.int16, oracle.layered_i16, 256)}[fmt]
    assert g + 2 * ((3 * g) >> 2) > qmax
    dv = H.sum(0).astype(np.int64)
    for k in (2, 3, 5):
        r = run(H, s, np.full(2, g, dt), 16, max_iters=k, early_stop=False)
        want = (g + dv * ((3 * qmax) >> 2)).astype(np.float32)
        assert np.array_equal(r.Q[0] * scale, want) and np.array_equal(r.Q[1] * scale, want)
        clamped_reading = np.float32(qmax + ((3 * qmax) >> 2))
        assert not np.any(r.Q[0] * scale == clamped_reading)


def _numpy_fx_layered(H, s, prior_bits, layer_size, max_iters, qmax, anum=3, ash=2, exact_q=True):
    """Independent layered fixed-point decoder: for each check of a layer,
    q = clamp(Q - r_old), the new r from (min1, min2) of |q| and the sign
    parity, then Q <- (Q - r_old) + r_new in exact integers (exact_q=False:
    Q <- q + r_new, the rejected reading).  Returns e, iterations, Q and the
    number of check inputs that saturated."""
    m, n = H.shape
    rows = [np.nonzero(H[i])[0] for i in range(m)]
    B = s.shape[0]
    out_e = np.zeros((B, n), np.uint8)
    out_it = np.zeros(B, np.int32)
    out_Q = np.zeros((B, n), np.int64)
    saturated = 0
    for b in range(B):
        r = [np.zeros(len(cc), np.int64) for cc in rows]
        Q = prior_bits[b].astype(np.int64).copy()
        for k in range(1, max_iters + 1):
            for lo in range(0, m, layer_size):
                for i in range(lo, lo + layer_size):
                    cc = rows[i]
                    x = Q[cc] - r[i]
                    q = np.clip(x, -qmax, qmax)
                    saturated += int(np.count_nonzero(q != x))
                    a = np.abs(q)
                    o = np.argsort(a, kind="stable")
                    m1, m2 = a[o[0]], a[o[1]]
                    neg = (q < 0).astype(np.int64)
                    par = (int(neg.sum()) + int(s[b, i])) & 1
                    mag = np.where(np.arange(len(cc)) == o[0], m2, m1)
                    rn = (1 - 2 * (par ^ neg)) * ((anum * mag) >> ash)
                    Q[cc] = (x + rn) if exact_q else (q + rn)
                    r[i] = rn
            e = (Q < 0).astype(np.uint8)
            if np.array_equal((e.astype(int) @ H.T) % 2, s[b]):
                break
        out_e[b], out_it[b], out_Q[b] = e, k, Q
    return out_e, out_it, out_Q, saturated


@pytest.mark.parametrize("fmt", ["i8", "i16"])
def test_layered_fixed_point_against_independent_decoder_saturating(fmt):
    """Per-bit priors of large magnitude (most at or near the bound, the
    error bits' priors pointing the wrong way half of the time), so the
    saturation branch of the layered rule decides many check inputs."""
    c = lp.lp_code(16)
    H = c.hz.dense()
    b = noise.Batch(c.hz, 31, np.arange(16), 0.06)
    rng = np.random.default_rng(77)
    qmax, dt, run, scale = {
        "i8": (127, np.int8, oracle.layered_i8, 16),
        "i16": (32767, np.int16, oracle.layered_i16, 256)}[fmt]
    mag = rng.integers(qmax // 3, qmax + 1, size=(b.B, c.n))
    wrong = (b.e == 1) & (rng.random((b.B, c.n)) < 0.5)
    prior = np.where(wrong, -mag, mag).astype(dt)
    r = run(H, b.s, prior, 16, max_iters=10)
    e, it, Q, sat = _numpy_fx_layered(H, b.s, prior, 16, 10, qmax)
    assert sat > 1000
    assert np.array_equal(r.e, e) and np.array_equal(r.iters, it)
    assert np.array_equal(r.Q * scale, Q.astype(np.float32))
    # the rejected reading (posterior rebuilt from the saturated input) is
    # told apart by this input
    e2, it2, Q2, _ = _numpy_fx_layered(H, b.s, prior, 16, 10, qmax, exact_q=False)
    assert not (np.array_equal(Q2, Q) and np.array_equal(it2, it))
