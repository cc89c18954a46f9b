"""Philox4x64-10 and the integer measurement matrix Q drawn from it.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.

Philox is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  One call maps a
4 x 64-bit counter and a 2 x 64-bit key to four 64-bit words through ten
rounds.  Each round takes the two 64x64->128-bit products of the multipliers
with counter words 0 and 2, and outputs
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0));
the key is advanced by the two Weyl increments before every round but the
first.

Measurement matrix (the paper asks only for a random Gaussian matrix,
Sections 1, 3.1 and 4): entry (i, j) of the M x n integer matrix Q takes word (i*n+j) mod 4 of
philox(counter=((i*n+j) div 4, n, 0, 0), key=(phi_seed, stream_id)) and sets
Q_ij = popcount(word) - 32, a Binomial(64, 1/2) - 32 variable in [-32, 32]:
mean 0, variance 16, excess kurtosis -1/32.  Phi = Q / (4 sqrt(M)) then has
variance 1/M per entry.  Rows are nested: Q for M rows is the row prefix of Q
for any M' > M.
"""
from __future__ import annotations

import numpy as np

MULT0 = 0xD2E7470EE14C6C93
MULT1 = 0xCA5A826395121157
WEYL0 = 0x9E3779B97F4A7C15
WEYL1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1


def philox4x64_10_scalar(ctr, key):
    """Reference round function on Python integers (one counter)."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in ctr)
    k0, k1 = (int(x) & MASK64 for x in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + WEYL0) & MASK64
            k1 = (k1 + WEYL1) & MASK64
        p0 = MULT0 * c0
        p1 = MULT1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & MASK64)
    return c0, c1, c2, c3


def _mulhilo(a: np.ndarray, b: int):
    """(hi, lo) 64-bit halves of a*b for a uint64 array and a 64-bit int."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo = a & m32
    a_hi = a >> s32
    b_lo = np.uint64(b & 0xFFFFFFFF)
    b_hi = np.uint64(b >> 32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    lo = a * np.uint64(b)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x64-10 over uint64 counter arrays (same key)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64).copy() for x in (c0, c1, c2, c3))
    for r in range(10):
        if r > 0:
            k0 = (k0 + WEYL0) & MASK64
            k1 = (k1 + WEYL1) & MASK64
        hi0, lo0 = _mulhilo(c0, MULT0)
        hi1, lo1 = _mulhilo(c2, MULT1)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def measurement_matrix_q(m: int, n: int, phi_seed: int, stream_id: int) -> np.ndarray:
    """Integer matrix Q (m x n, int64 values in [-32, 32])."""
    total = m * n
    n_ctr = (total + 3) // 4
    ctr = np.arange(n_ctr, dtype=np.uint64)
    zeros = np.zeros(n_ctr, dtype=np.uint64)
    w = philox4x64_10(ctr, np.full(n_ctr, n, dtype=np.uint64), zeros, zeros,
                      int(phi_seed) & MASK64, int(stream_id) & MASK64)
    words = np.stack(w, axis=1).reshape(-1)[:total]
    q = np.bitwise_count(words).astype(np.int64) - 32
    return q.reshape(m, n)


def phi_scale(m: int) -> float:
    """s_Phi = 1 / (4 sqrt(M)), so that Phi = s_Phi * Q has variance 1/M."""
    return 1.0 / (4.0 * np.sqrt(m))


def measurement_rows_q(rows, n: int, phi_seed: int, stream_id: int) -> np.ndarray:
    """Selected rows of Q (len(rows) x n) with the same entries as
    `measurement_matrix_q`: entry (i, j) is word (i n + j) mod 4 of the
    Philox block at counter (i n + j) div 4."""
    rows = np.asarray(rows, dtype=np.int64)
    idx = (rows[:, None] * n + np.arange(n, dtype=np.int64)[None, :]).reshape(-1)
    ctr = (idx // 4).astype(np.uint64)
    zeros = np.zeros_like(ctr)
    w = philox4x64_10(ctr, np.full(ctr.shape, n, dtype=np.uint64), zeros, zeros,
                      int(phi_seed) & MASK64, int(stream_id) & MASK64)
    words = np.stack(w, axis=1)[np.arange(idx.size), idx % 4]
    q = np.bitwise_count(words).astype(np.int64) - 32
    return q.reshape(rows.size, n)
