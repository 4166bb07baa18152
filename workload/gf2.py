"""GF(2) linear algebra for evaluating decodes (not part of decoding).

A decode of the H_Z side fails logically when the residual rho = e xor e_hat
anticommutes with a logical Z operator.  Logical Z operators are ker(H_X)
modulo rowspace(H_Z) (stabilizers commute, CSS condition of Section 2); a
basis Lambda_Z has k = n - rank H_X - rank H_Z rows.  A shot fails iff the
decoder did not converge or Lambda_Z rho^T != 0.

Rows are packed into uint64 words (bit j of row -> word j // 64, bit j % 64)
so elimination is a few thousand vectorised XORs even at n = 4352.
"""
from __future__ import annotations

import numpy as np


def pack_rows(h: np.ndarray) -> np.ndarray:
    h = np.asarray(h, dtype=np.uint8)
    m, n = h.shape
    w = (n + 63) // 64
    pad = np.zeros((m, w * 64), dtype=np.uint8)
    pad[:, :n] = h & 1
    by = np.packbits(pad.reshape(m, w * 8, 8), axis=2, bitorder="little").reshape(m, w * 8)
    return by.view("<u8").reshape(m, w).copy()


def unpack_rows(p: np.ndarray, n: int) -> np.ndarray:
    p = np.ascontiguousarray(p.astype("<u8"))
    by = p.view(np.uint8).reshape(p.shape[0], -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :n].copy()


def _bit(p: np.ndarray, j: int) -> np.ndarray:
    return (p[:, j >> 6] >> np.uint64(j & 63)) & np.uint64(1)


def rref(h: np.ndarray):
    """Reduced row echelon form over GF(2). Returns (packed rows, pivot cols)."""
    h = np.asarray(h, dtype=np.uint8)
    n = h.shape[1]
    p = pack_rows(h)
    pivots = []
    r = 0
    for c in range(n):
        if r == p.shape[0]:
            break
        col = _bit(p[r:], c).astype(bool)
        nz = np.nonzero(col)[0]
        if nz.size == 0:
            continue
        k = r + nz[0]
        if k != r:
            p[[r, k]] = p[[k, r]]
        hit = _bit(p, c).astype(bool)
        hit[r] = False
        p[hit] ^= p[r]
        pivots.append(c)
        r += 1
    return p[:r], pivots


def rank(h: np.ndarray) -> int:
    return len(rref(h)[1])


def kernel(h: np.ndarray) -> np.ndarray:
    """Basis of {x : h x^T = 0} as uint8 rows."""
    h = np.asarray(h, dtype=np.uint8)
    n = h.shape[1]
    red, piv = rref(h)
    dense = unpack_rows(red, n)
    free = [c for c in range(n) if c not in set(piv)]
    basis = np.zeros((len(free), n), dtype=np.uint8)
    for i, f in enumerate(free):
        basis[i, f] = 1
        for r, pc in enumerate(piv):
            basis[i, pc] = dense[r, f]
    return basis


def logical_basis(hx: np.ndarray, hz: np.ndarray) -> np.ndarray:
    """Lambda_Z: rows of ker(H_X) independent modulo rowspace(H_Z).

    The running basis is kept fully reduced (each pivot column set in exactly
    one row), so reducing a vector is one XOR of the rows whose pivot bits it
    has.
    """
    hx = np.asarray(hx, dtype=np.uint8)
    hz = np.asarray(hz, dtype=np.uint8)
    n = hx.shape[1]
    ker = pack_rows(kernel(hx))
    red, piv = rref(hz)
    rows = [r for r in red]
    pivs = list(piv)
    keep_idx = []
    for v in ker:
        if rows:
            R = np.array(rows)
            P = np.array(pivs)
            sel = ((v[P >> 6] >> (P & 63).astype(np.uint64)) & np.uint64(1)).astype(bool)
            if sel.any():
                v = v ^ np.bitwise_xor.reduce(R[sel], axis=0)
        nzw = np.nonzero(v)[0]
        if nzw.size == 0:
            continue
        w0 = int(nzw[0])
        low = int(v[w0] & (~v[w0] + np.uint64(1)))
        pc = w0 * 64 + low.bit_length() - 1
        for i in range(len(rows)):
            if (rows[i][pc >> 6] >> np.uint64(pc & 63)) & np.uint64(1):
                rows[i] = rows[i] ^ v
        rows.append(v)
        pivs.append(pc)
        keep_idx.append(len(rows) - 1)
    if not keep_idx:
        return np.zeros((0, n), dtype=np.uint8)
    return unpack_rows(np.array([rows[i] for i in keep_idx]), n)


def parity_rows(rows_packed: np.ndarray, x: np.ndarray) -> np.ndarray:
    """[B, k] parities <row_i, x_b> for uint8 x [B, n] (rows packed uint64)."""
    xp = pack_rows(x)
    out = np.zeros((x.shape[0], rows_packed.shape[0]), dtype=np.uint8)
    for i, row in enumerate(rows_packed):
        acc = np.bitwise_xor.reduce(xp & row[None, :], axis=1)
        # parity of a uint64 via folding
        for sh in (32, 16, 8, 4, 2, 1):
            acc ^= acc >> np.uint64(sh)
        out[:, i] = (acc & np.uint64(1)).astype(np.uint8)
    return out


def logical_failures(lam: np.ndarray, e: np.ndarray, e_hat: np.ndarray,
                     converged: np.ndarray) -> np.ndarray:
    """bool [B]: not converged, or the residual flips some logical."""
    rho = (np.asarray(e, dtype=np.uint8) ^ np.asarray(e_hat, dtype=np.uint8))
    flips = parity_rows(pack_rows(lam), rho).any(axis=1)
    return flips | (np.asarray(converged) == 0)


def wilson(k: int, n: int, z: float = 1.96):
    """Wilson score interval for a binomial rate k/n."""
    if n == 0:
        return (0.0, 1.0)
    ph = k / n
    d = 1 + z * z / n
    c = (ph + z * z / (2 * n)) / d
    h = z * np.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))
