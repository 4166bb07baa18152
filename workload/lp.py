"""Lifted-product CSS codes LP(A, A*) over F2[x]/(x^L - 1).

The decoder's inputs are the parity-check matrices of a CSS code: H_X and
H_Z must commute (H_X H_Z^T = 0 over GF(2), CSS condition of Section 2) and
the X-error syndrome is s = H_Z e^T.  The workloads use the lifted-product
family (Panteleev and Kalachev, cited in Section 1):

* A is a 3 x 5 matrix whose entries are monomials x^a, a uniform in [0, L),
  drawn from the counter-based generator with key (2508, 7879, L).
* A* is the conjugate transpose: A*[j][i] = x^(-a_ij mod L).
* H_X = [A (x) I_5 | I_3 (x) A*] and H_Z = [I_5 (x) A | A* (x) I_3], each
  15 x 34 blocks of L x L circulants: N = 34L qubits, M = 15L checks.
* A monomial x^a is the circulant P^a with P^a[r][(r + a) mod L] = 1.
* Kronecker index (i, k) of X (x) Y maps to i * dim(Y) + k.

H_X H_Z^T = A (x) A* + A (x) A* = 0 because the group ring is commutative.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import rng

LP_SEED = (2508, 7879)   # the workload's code seed; the third key part is L
BASE_M, BASE_N = 3, 5


def base_exponents(L: int, seed: tuple = LP_SEED) -> np.ndarray:
    """3 x 5 exponent matrix of A, each entry uniform in [0, L)."""
    s = (seed[0] << 32) ^ (seed[1] << 8) ^ L
    d = rng.draws(s, rng.DOMAIN_CODE, np.arange(BASE_M)[:, None], np.arange(BASE_N)[None, :])
    return (d % np.uint64(L)).astype(np.int64)


def lp_block_tables(a: np.ndarray, L: int):
    """Base exponent tables (-1 = zero block) of H_X and H_Z, each 15 x 34."""
    ma, na = a.shape
    off = na * na                     # 25 left block columns
    nb = off + ma * ma                # + 9 right block columns
    mb = ma * na                      # 15 block rows
    hx = -np.ones((mb, nb), dtype=np.int64)
    hz = -np.ones((mb, nb), dtype=np.int64)
    astar = lambda j, i: (-a[i, j]) % L          # A*[j][i]
    # H_X left: A (x) I_na, rows (i,k) -> i*na+k, cols (j,l) -> j*na+l, delta_kl
    for i in range(ma):
        for j in range(na):
            for k in range(na):
                hx[i * na + k, j * na + k] = a[i, j]
    # H_X right: I_ma (x) A*, rows (b, c) -> b*na + c, cols (d, e) -> off + d*ma + e, delta_bd
    for b in range(ma):
        for c in range(na):
            for e in range(ma):
                hx[b * na + c, off + b * ma + e] = astar(c, e)
    # H_Z left: I_na (x) A, rows (k,i) -> k*ma+i, cols (l,j) -> l*na+j, delta_kl
    for k in range(na):
        for i in range(ma):
            for j in range(na):
                hz[k * ma + i, k * na + j] = a[i, j]
    # H_Z right: A* (x) I_ma, rows (c, b) -> c*ma+b, cols (e, d) -> off + e*ma + d, delta_bd
    for c in range(na):
        for b in range(ma):
            for e in range(ma):
                hz[c * ma + b, off + e * ma + b] = astar(c, e)
    return hx, hz


def expand_csr(base: np.ndarray, L: int):
    """CSR (row_ptr, col_idx) of the lifted matrix; columns increase per row."""
    mb, nb = base.shape
    rows = []
    for R in range(mb):
        blocks = [(C, int(base[R, C])) for C in range(nb) if base[R, C] >= 0]
        for r in range(L):
            rows.append(sorted(C * L + (r + s) % L for C, s in blocks))
    row_ptr = np.zeros(mb * L + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum([len(c) for c in rows])
    col_idx = np.array([c for cs in rows for c in cs], dtype=np.int32)
    return row_ptr, col_idx


def csr_to_dense(m: int, n: int, row_ptr, col_idx) -> np.ndarray:
    h = np.zeros((m, n), dtype=np.uint8)
    for r in range(m):
        h[r, col_idx[row_ptr[r]:row_ptr[r + 1]]] = 1
    return h


@dataclass
class Side:
    """One CSS side: the matrix whose syndrome a decoder consumes."""
    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    lift: int = 0
    base: np.ndarray | None = None    # base_m x base_n exponents, -1 = zero

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        return csr_to_dense(self.m, self.n, self.row_ptr, self.col_idx)


@dataclass
class LPCode:
    L: int
    a: np.ndarray
    hx: Side
    hz: Side
    n: int = field(init=False)

    def __post_init__(self):
        self.n = self.hz.n


def lp_code(L: int, seed: tuple = LP_SEED) -> LPCode:
    a = base_exponents(L, seed)
    bx, bz = lp_block_tables(a, L)
    sides = []
    for base in (bx, bz):
        rp, ci = expand_csr(base, L)
        sides.append(Side(base.shape[0] * L, base.shape[1] * L, rp, ci, L, base))
    return LPCode(L, a, sides[0], sides[1])


def side_from_dense(h: np.ndarray) -> Side:
    h = np.asarray(h, dtype=np.uint8)
    m, n = h.shape
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    cols = []
    for r in range(m):
        c = np.nonzero(h[r])[0]
        cols.extend(c.tolist())
        row_ptr[r + 1] = len(cols)
    return Side(m, n, row_ptr, np.array(cols, dtype=np.int32))
